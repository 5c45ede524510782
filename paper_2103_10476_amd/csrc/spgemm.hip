// Sparse matrix-matrix product C = X*Y for the Galerkin operator (Sec. 1.1), in Gustavson
// order: every output entry C_ij accumulates X_ik*Y_kj over the row's entries k in ascending
// order, from 0.  No floating-point atomics: each output row's products are either ordered by
// (column, position), every run of equal columns summed in order by one lane, or added X entry
// by X entry, in order, to per-column accumulators of one wavefront.  Output rows are sorted;
// cancellations stay stored.
//
// Rows are binned by their product count T:
//   T <= 64      8, 16 or 32 lanes per row (8, 4 or 2 rows per wavefront): two products per
//                lane, rank sort in LDS;
//   T <= 256     one wavefront per row, 64 products per step sorted in registers, each run
//                added to its column's sum in an LDS hash table;
//   T <= 1024    one 256-thread block per row: the row's products sorted by (column,
//                position) in LDS, each run reduced in order and written at its rank; for
//                R (A P) the rank accumulator (k_esc_rank) takes these rows first;
//   T > 1024     the row's dense column window in LDS when the output width fits (products
//                taken 64 per step and sorted, or, for long Y rows, one X entry per step with
//                its Y row across the lanes), else the wavefront kernel with a 2048-slot
//                hash table;
//   hash > 1/2   long rows with more than 1024 distinct columns are redone over their column
//                windows in LDS tiles (one launch per tile, up to 8), or with a dense
//                accumulator in global memory when the windows need more tiles.
// Results go to per-row slots at the row's product offset (room for T >= distinct entries)
// and are compacted into CSR afterwards.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>

#include <mutex>

#include "kernels.hpp"

namespace sa {

constexpr int kWave = 64;
constexpr int kChunk = 1024;  // products per block-level chunk

// Bins by product count: <= 16, <= 32, <= 64 (rows sharing wavefronts), <= 256, <= 1024
// (block per row, one chunk), longer.
constexpr int kBins = 6;
__device__ __forceinline__ int bin_of(int64_t T) {
  return T <= 16 ? 0 : T <= 32 ? 1 : T <= kWave ? 2 : T <= 256 ? 3 : T <= kChunk ? 4 : 5;
}

// A block lists its rows per bin: counted in LDS, each non-empty bin's share reserved with one
// global atomic (the order inside a list is immaterial: rows are independent).
__device__ __forceinline__ void bin_row(bool live, int32_t i, int64_t T, int32_t m,
                                        int32_t *lists, int32_t *counters) {
  __shared__ int32_t s_cnt[kBins], s_base[kBins];
  if (threadIdx.x < kBins) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const int bin = bin_of(T);
  int32_t local = 0;
  if (live) local = atomicAdd(&s_cnt[bin], 1);
  __syncthreads();
  if (threadIdx.x < kBins && s_cnt[threadIdx.x] > 0)
    s_base[threadIdx.x] = atomicAdd(&counters[threadIdx.x], s_cnt[threadIdx.x]);
  __syncthreads();
  if (live) lists[(int64_t)bin * m + s_base[bin] + local] = i;
}

// Thread per row of X: the row's product count T, the products before each of its entries
// (xpref), and the row's place in its bin's list.  The block's prefixes are gathered in LDS
// and written out as one contiguous run (a thread's own entries are a short strided run, whose
// partial-line writes cost several times their bytes), unless the block's X entries exceed
// the buffer.
constexpr int32_t kCountLds = 4096;
__global__ __launch_bounds__(kBlock) void k_count_products(int32_t m, const int32_t *xrp,
                                                           const int32_t *xcol,
                                                           const int32_t *yrp, int64_t *cnt,
                                                           int32_t *xpref, int32_t *lists,
                                                           int32_t *counters) {
  __shared__ int32_t s_xp[kCountLds];
  const int64_t r0 = (int64_t)blockIdx.x * blockDim.x;
  const int32_t e0 = xrp[r0], e1 = xrp[min((int64_t)m, r0 + blockDim.x)];
  const bool staged = e1 - e0 <= kCountLds;  // block-uniform
  const int64_t i64 = r0 + threadIdx.x;
  const bool live = i64 < m;
  const int32_t i = live ? (int32_t)i64 : 0;
  int64_t t = 0;
  if (live) {
    for (int32_t e = xrp[i]; e < xrp[i + 1]; ++e) {
      // products before entry e within the row (T < 2^31 checked)
      if (staged) s_xp[e - e0] = (int32_t)t;
      else xpref[e] = (int32_t)t;
      const int32_t k = xcol[e];
      t += yrp[k + 1] - yrp[k];
    }
    cnt[i] = t;
  }
  bin_row(live, i, t, m, lists, counters);  // every thread passes the barriers
  if (staged) {
    __syncthreads();
    for (int32_t q = threadIdx.x; q < e1 - e0; q += blockDim.x) xpref[e0 + q] = s_xp[q];
  }
}

// One wavefront per row of X (long rows): xpref by a wavefront prefix sum.
__global__ __launch_bounds__(64) void k_count_products_w(int32_t m, const int32_t *xrp,
                                                         const int32_t *xcol,
                                                         const int32_t *yrp, int64_t *cnt,
                                                         int32_t *xpref) {
  const int32_t i = blockIdx.x;
  if (i >= m) return;
  const int lane = threadIdx.x;
  int64_t base = 0;
  for (int32_t c = xrp[i]; c < xrp[i + 1]; c += 64) {
    const int32_t e = c + lane;
    int32_t len = 0;
    if (e < xrp[i + 1]) {
      const int32_t k = xcol[e];
      len = yrp[k + 1] - yrp[k];
    }
    int32_t incl = len;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (e < xrp[i + 1]) xpref[e] = (int32_t)(base + incl - len);
    base += __shfl(incl, 63, 64);
  }
  if (lane == 0) cnt[i] = base;
}

// ---- G lanes per row (T <= G P), 64/G rows per wavefront -----------------------------------
// A wavefront takes 64/G rows, G lanes each, P products per lane: short rows share a
// wavefront instead of leaving most of its lanes idle, and the more rows a wavefront holds,
// the more of their (dependent) loads are in flight together.  Per row: the X entries G at a
// time (a segmented scan of their Y-row lengths), the products by binary search over the scan
// (lane l takes products l, l+G, ...), a rank sort of the T <= G P products in LDS by
// (column, position), and one lane per run of equal columns summing it in order.  The chunk
// loop runs to the longest X row of the wavefront, so every lane passes every barrier.
template <int G, int P>
__global__ __launch_bounds__(kWave) void k_esc_group(
    const int32_t *rows, int32_t nrows, const int32_t *xrp, const int32_t *xcol,
    const double *xval, const int32_t *yrp, const int32_t *ycol, const double *yval,
    const int64_t *poff, int32_t *ocol, double *oval, int32_t *ucnt) {
  static_assert((G == 8 || G == 16 || G == 32 || G == 64) && (P == 1 || P == 2),
                "group width, products per lane");
  constexpr int CAP = G * P;  // products of one row at most
  __shared__ int32_t keys[kWave * P];
  __shared__ double vals[kWave * P];
  __shared__ int32_t skeys[kWave * P];
  __shared__ double svals[kWave * P];
  __shared__ int32_t s_incl[kWave], s_ys[kWave];
  __shared__ double s_a[kWave];
  const int lane = threadIdx.x;
  const int gl = lane % G, gb = lane - gl;  // lane in the group, the group's first lane
  const int pb = (lane / G) * CAP;          // the row's product slots in keys/vals
  // consecutive rows share the Y rows of their neighbours: each XCD takes a contiguous run of
  // the bin's rows (bins list rows roughly in row order), so those reads hit its L2
  const int64_t r64 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kWave / G) + lane / G;
  const bool live = r64 < nrows;
  const int32_t i = live ? rows[r64] : 0;
  const int64_t base = live ? poff[i] : 0;
  const int32_t T = live ? (int32_t)(poff[i + 1] - base) : 0;
  const int32_t xb = live ? xrp[i] : 0, xe = live ? xrp[i + 1] : 0;
  int32_t nch = (xe - xb + G - 1) / G;  // chunks of this row; the wavefront runs the most
  for (int off = 32; off >= 1; off >>= 1) nch = max(nch, __shfl_xor(nch, off, kWave));
  // expansion in Gustavson order: position = products of earlier X entries + offset in Y row
  int32_t filled = 0;
  for (int32_t c = 0; c < nch; ++c) {
    const int32_t e = xb + c * G + gl;
    int32_t len = 0, ys = 0;
    double a = 0.0;
    if (e < xe) {
      const int32_t k = xcol[e];
      a = xval[e];
      ys = yrp[k];
      len = yrp[k + 1] - ys;
    }
    // inclusive scan of len within the group
    int32_t incl = len;
    for (int off = 1; off < G; off <<= 1) {
      const int32_t v = __shfl_up(incl, off, G);
      if (gl >= off) incl += v;
    }
    const int32_t tot = __shfl(incl, G - 1, G);
    s_incl[lane] = incl;
    s_ys[lane] = ys;
    s_a[lane] = a;
    __syncthreads();
    // product p of this chunk comes from the first entry s with incl[s] > p, at offset
    // p - incl[s-1] in its row of Y: loads independent across lanes.  A lane's products are
    // gl, gl + G, ... (at most P, since tot <= T <= G P): all are located first, then their
    // loads issued together
    int32_t qu[P], su[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int32_t p = gl + u * G;
      su[u] = -1;
      if (p < tot) {
        int32_t lo = 0, hi = G - 1;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (s_incl[gb + mid] > p) hi = mid;
          else lo = mid + 1;
        }
        su[u] = lo;
        qu[u] = s_ys[gb + lo] + p - (lo > 0 ? s_incl[gb + lo - 1] : 0);
      }
    }
    int32_t cu[P];
    double yu[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (su[u] >= 0) {
        cu[u] = ycol[qu[u]];
        yu[u] = yval[qu[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (su[u] >= 0) {
        const int32_t p = gl + u * G;
        keys[pb + filled + p] = cu[u];
        vals[pb + filled + p] = s_a[gb + su[u]] * yu[u];
      }
    }
    __syncthreads();
    filled += tot;
  }
  // rank sort: positions q G + gl of the row, ordered by (column, position)
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int32_t pos = q * G + gl;
    if (pos < T) {
      const int32_t key = keys[pb + pos];
      int32_t rank = 0;
      for (int32_t r = 0; r < T; ++r) {
        const int32_t kr = keys[pb + r];
        rank += (kr < key) || (kr == key && r < pos);
      }
      skeys[pb + rank] = key;
      svals[pb + rank] = vals[pb + pos];
    }
  }
  __syncthreads();
  // one lane per run of equal columns adds it in order from 0 and writes it at the run's rank
  int32_t before = 0;  // runs in the earlier position slices of the row
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int32_t pos = q * G + gl;
    bool head = false;
    int32_t key = 0;
    double sum = 0.0;
    if (pos < T) {
      key = skeys[pb + pos];
      head = (pos == 0) || (skeys[pb + pos - 1] != key);
      if (head)
        for (int32_t r = pos; r < T && skeys[pb + r] == key; ++r) sum += svals[pb + r];
    }
    const unsigned long long gm =
        (__ballot(head) >> gb) & (~0ull >> (64 - G));  // this group's heads in slice q
    const int32_t idx = before + __popcll(gm & ((1ull << gl) - 1ull));
    if (head) {
      ocol[base + idx] = key;
      oval[base + idx] = sum;
    }
    before += __popcll(gm);
  }
  if (live && gl == 0) ucnt[i] = before;
}

// ---- block-level rows (T > 64) -------------------------------------------------------------
__device__ inline int32_t find_entry(const int32_t *xpref, int32_t xb, int32_t xe, int32_t p) {
  // last e in [xb, xe) with xpref[e] <= p (entries with no products share a prefix value;
  // the last one holding p is the one whose Y row contains it).
  int32_t lo = xb, hi = xe - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (xpref[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ inline void bitonic_u64(uint64_t *a, int32_t L) {
  for (int32_t k = 2; k <= L; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t idx = threadIdx.x; idx < L; idx += blockDim.x) {
        const int32_t ixj = idx ^ j;
        if (ixj > idx) {
          const uint64_t x = a[idx], y = a[ixj];
          const bool up = (idx & k) == 0;
          if ((x > y) == up) {
            a[idx] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ inline int32_t next_pow2(int32_t x) {
  int32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

__device__ inline uint32_t hash_slot(int32_t key, uint32_t mask) {
  return ((uint32_t)key * 2654435761u) & mask;
}

// Loads products c0 .. c0+L-1 of row i into sk (column << 32 | position) / sv and sorts sk;
// after it, equal columns are adjacent in position (= Gustavson) order.
__device__ inline void load_sorted_chunk(int32_t c0, int32_t L, int32_t xb, int32_t xe,
                                         const int32_t *xpref, const int32_t *xcol,
                                         const double *xval, const int32_t *yrp,
                                         const int32_t *ycol, const double *yval, uint64_t *sk,
                                         double *sv) {
  const int32_t Lp = next_pow2(L);
  for (int32_t q = threadIdx.x; q < Lp; q += blockDim.x) {
    if (q < L) {
      const int32_t p = c0 + q;
      const int32_t e = find_entry(xpref, xb, xe, p);
      const int32_t k = xcol[e];
      const int32_t yy = yrp[k] + (p - xpref[e]);
      sk[q] = ((uint64_t)(uint32_t)ycol[yy] << 32) | (uint32_t)q;
      sv[q] = xval[e] * yval[yy];
    } else {
      sk[q] = ~0ull;
    }
  }
  __syncthreads();
  bitonic_u64(sk, Lp);
}

__device__ inline uint32_t key_of(uint64_t x) { return (uint32_t)(x >> 32); }

// Single chunk: T <= 4*BS products, one block of BS threads per row; each run of equal columns
// is summed in position order by its first lane and written at the run's rank.
template <int BS>
__global__ __launch_bounds__(BS) void k_esc_single(
    const int32_t *rows, int32_t nrows, const int32_t *xrp, const int32_t *xcol,
    const double *xval, const int32_t *xpref, const int32_t *yrp, const int32_t *ycol,
    const double *yval, const int64_t *poff, int32_t *ocol, double *oval, int32_t *ucnt,
    const int32_t *dcount) {
  constexpr int CH = 4 * BS;
  __shared__ uint64_t sk[CH];
  __shared__ double sv[CH];
  __shared__ int32_t s_scan[BS];
  const int tid = threadIdx.x;
  const int32_t slot = blockIdx.x;
  if (slot >= (dcount ? *dcount : nrows)) return;  // block-uniform
  const int32_t i = rows[slot];
  const int64_t base = poff[i];
  const int32_t L = (int32_t)(poff[i + 1] - base);
  load_sorted_chunk(0, L, xrp[i], xrp[i + 1], xpref, xcol, xval, yrp, ycol, yval, sk, sv);
  int32_t nh = 0;
  for (int32_t r = tid * 4; r < tid * 4 + 4; ++r)
    if (r < L && (r == 0 || key_of(sk[r]) != key_of(sk[r - 1]))) ++nh;
  s_scan[tid] = nh;
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    const int32_t add = (tid >= off) ? s_scan[tid - off] : 0;
    __syncthreads();
    s_scan[tid] += add;
    __syncthreads();
  }
  int32_t idx = s_scan[tid] - nh;
  for (int32_t r = tid * 4; r < tid * 4 + 4; ++r) {
    if (r < L && (r == 0 || key_of(sk[r]) != key_of(sk[r - 1]))) {
      const uint32_t key = key_of(sk[r]);
      double sum = 0.0;
      for (int32_t q = r; q < L && key_of(sk[q]) == key; ++q) sum += sv[(uint32_t)sk[q]];
      ocol[base + idx] = (int32_t)key;
      oval[base + idx] = sum;
      ++idx;
    }
  }
  if (tid == BS - 1) ucnt[i] = s_scan[BS - 1];
}

// Rows with more distinct columns than the LDS table holds, when their column windows need
// more LDS tiles than the limit: a dense accumulator of ncols entries per block in global
// memory (first touch starts from 0, adds in position order as above); the result is
// extracted in column order by a block-wide scan of the touched flags.
__global__ __launch_bounds__(kBlock) void k_esc_dense(
    const int32_t *rows, int32_t nrows, const int32_t *xrp, const int32_t *xcol,
    const double *xval, const int32_t *xpref, const int32_t *yrp, const int32_t *ycol,
    const double *yval, int32_t ncols, const int64_t *poff, int32_t *ocol, double *oval,
    int32_t *ucnt, double *dacc, int32_t *dflag) {
  __shared__ uint64_t sk[kChunk];
  __shared__ double sv[kChunk];
  __shared__ int32_t s_scan[kBlock];
  __shared__ int32_t s_base;
  const int tid = threadIdx.x;
  double *acc = dacc + (int64_t)blockIdx.x * ncols;
  int32_t *flag = dflag + (int64_t)blockIdx.x * ncols;
  for (int32_t slot = blockIdx.x; slot < nrows; slot += gridDim.x) {
    const int32_t i = rows[slot];
    const int32_t xb = xrp[i], xe = xrp[i + 1];
    const int64_t base = poff[i];
    const int32_t T = (int32_t)(poff[i + 1] - base);
    for (int32_t q = tid; q < ncols; q += kBlock) flag[q] = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < T; c0 += kChunk) {
      const int32_t L = min(kChunk, T - c0);
      load_sorted_chunk(c0, L, xb, xe, xpref, xcol, xval, yrp, ycol, yval, sk, sv);
      for (int32_t r = tid; r < L; r += kBlock) {
        const uint32_t key = key_of(sk[r]);
        if (r > 0 && key_of(sk[r - 1]) == key) continue;
        double a = flag[key] ? acc[key] : 0.0;
        for (int32_t q = r; q < L && key_of(sk[q]) == key; ++q) a += sv[(uint32_t)sk[q]];
        acc[key] = a;
        flag[key] = 1;
      }
      __syncthreads();
    }
    if (tid == 0) s_base = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < ncols; c0 += kBlock) {
      const int32_t c = c0 + tid;
      const int32_t f = (c < ncols) ? flag[c] : 0;
      s_scan[tid] = f;
      __syncthreads();
      for (int off = 1; off < kBlock; off <<= 1) {
        const int32_t add = (tid >= off) ? s_scan[tid - off] : 0;
        __syncthreads();
        s_scan[tid] += add;
        __syncthreads();
      }
      if (f) {
        const int32_t pos = s_base + s_scan[tid] - 1;
        ocol[base + pos] = c;
        oval[base + pos] = acc[c];
      }
      __syncthreads();
      if (tid == kBlock - 1) s_base += s_scan[kBlock - 1];
      __syncthreads();
    }
    if (tid == 0) ucnt[i] = s_base;
    __syncthreads();
  }
}

// Long rows whose output columns fit in LDS (the dense coarse levels): one wavefront per row
// with a dense accumulator of ncols doubles and a touched-column bitmap in LDS.  The row's
// entries k are taken in ascending order; for each, the lanes add the products of Y's row k
// into their own columns (distinct within a row of Y), and the adds of successive k are
// ordered (one wavefront executes them in program order; a wave barrier separates them), so
// every output entry receives its products in ascending k from 0, as in the sort-based bins.
// The row's X entries and Y row ranges are staged in LDS 64 at a time, and the steps (64-entry
// slices of Y rows) are taken D at a time, their loads issued together before they are added,
// so D steps share one memory latency even at one wavefront per CU (the widest windows fill
// the LDS).
// The result is extracted in column order with ballots.  Rows wider than the LDS (those that
// overflow the hash bin) are taken in column tiles, one launch per tile, each appending its
// entries to the row's earlier ones.
__device__ __forceinline__ void lds_add(double *acc, uint32_t *bits, int32_t j, double v) {
  acc[j] = acc[j] + v;
  atomicOr(&bits[j >> 5], 1u << (j & 31));
}
// Column window of each long row (rows[slot]): from the smallest first column to the largest
// last column of the Y rows it touches (Y's rows are sorted, as every matrix the setup
// builds); win[slot] = (first column, width), and *maxw the largest width.
// One wavefront per row (X rows of the long bin reach thousands of entries): lanes take the
// row's entries, then a shuffle minimum / maximum.
__global__ void k_row_window(const int32_t *rows, int32_t nrows, const int32_t *xrp,
                             const int32_t *xcol, const int32_t *yrp, const int32_t *ycol,
                             int2 *win, int32_t *maxw) {
  const int64_t slot = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (slot >= nrows) return;  // wave-uniform
  const int lane = threadIdx.x & 63;
  const int32_t i = rows[slot];
  int32_t lo = 0x7fffffff, hi = -1;
  for (int32_t e = xrp[i] + lane; e < xrp[i + 1]; e += 64) {
    const int32_t k = xcol[e];
    const int32_t b = yrp[k], en = yrp[k + 1];
    if (b < en) {
      lo = min(lo, ycol[b]);
      hi = max(hi, ycol[en - 1]);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  if (lane == 0) {
    const int32_t w = hi >= lo ? hi - lo + 1 : 0;
    win[slot] = make_int2(hi >= lo ? lo : 0, w);
    atomicMax(maxw, w);
  }
}

constexpr int kLdsDepth = 8;  // steps whose loads k_esc_lds issues together
template <int D>
__global__ __launch_bounds__(64) void k_esc_lds(const int32_t *rows, int32_t nrows,
                                                const int32_t *xrp, const int32_t *xcol,
                                                const double *xval, const int32_t *yrp,
                                                const int32_t *ycol, const double *yval,
                                                int32_t ncols, const int2 *win,
                                                const int64_t *poff, int32_t *ocol,
                                                double *oval, int32_t *ucnt, int32_t tile,
                                                int32_t tw) {
  extern __shared__ double lds_acc[];
  double *acc = lds_acc;
  uint32_t *bits = (uint32_t *)(acc + ncols);
  __shared__ double s_a[64];
  __shared__ int32_t s_b[64], s_e[64];
  const int lane = threadIdx.x;
  const int32_t slot = blockIdx.x;
  if (slot >= nrows) return;  // block-uniform
  const int32_t i = rows[slot];
  // the row's window: accumulator index j - lo for output column j, rw <= ncols entries
  // (no windows: the whole width); with tiles (tw > 0) this pass takes columns
  // [lo + tile tw, lo + (tile + 1) tw) of the window and appends to the earlier tiles' entries
  const int2 wn = win ? win[slot] : make_int2(0, ncols);
  int32_t lo = wn.x, rw = wn.y, prior = 0;
  if (tw > 0) {
    const int32_t off = tile * tw;
    if (tile > 0 && off >= rw) return;  // block-uniform: the row's window ended earlier
    lo += off;
    rw = min(tw, rw - off);
    if (tile > 0) prior = ucnt[i];
  }
  const int32_t nw = (rw + 31) >> 5;
  for (int32_t c = lane; c < rw; c += 64) acc[c] = 0.0;
  for (int32_t c = lane; c < nw; c += 64) bits[c] = 0u;
  const int32_t xb = xrp[i], xe = xrp[i + 1];
  for (int32_t e0 = xb; e0 < xe; e0 += 64) {
    const int32_t cnt = min(64, xe - e0);
    __syncthreads();
    if (lane < cnt) {
      const int32_t k = xcol[e0 + lane];
      s_a[lane] = xval[e0 + lane];
      s_b[lane] = yrp[k];
      s_e[lane] = yrp[k + 1];
    }
    __syncthreads();
    // steps (g, 64-entry slice of Y's row k_g) in order, D at a time: the D steps' loads are
    // issued together, then the steps are added in order (steps past the chunk are empty).
    // Every lane loads (lanes past the Y row, or steps past the chunk, read the chunk's first
    // Y entry and discard it), so each step waits only for its own loads.  The block is one
    // wavefront, whose LDS operations complete in program order, and one step's adds go to
    // distinct columns (one Y row's): no barrier between steps, which would also wait for the
    // loads in flight.
    const int32_t qsafe = s_b[0] < s_e[0] ? s_b[0] : 0;
    int32_t gp = 0, qp = s_b[0];
    while (gp < cnt) {
      int32_t jq[D], gq[D];
      double vq[D];
      bool okq[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        gq[d] = gp;
        const bool live = gp < cnt;
        const int32_t ge = live ? s_e[gp] : 0;
        okq[d] = live && qp + lane < ge;
        const int32_t q = okq[d] ? qp + lane : qsafe;
        jq[d] = ycol[q];
        vq[d] = yval[q];
        if (live) {
          qp += 64;
          if (qp >= ge) {
            ++gp;
            qp = (gp < cnt) ? s_b[gp] : 0;
          }
        }
      }
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int32_t j = jq[d];
        if (okq[d] && (uint32_t)(j - lo) < (uint32_t)rw)
          lds_add(acc, bits, j - lo, s_a[gq[d]] * vq[d]);
      }
    }
  }
  __syncthreads();
  const int64_t base = poff[i] + prior;
  int32_t w = 0;
  for (int32_t c0 = 0; c0 < rw; c0 += 64) {
    const int32_t c = c0 + lane;
    const bool f = c < rw && ((bits[c >> 5] >> (c & 31)) & 1u);
    const unsigned long long bm = __ballot(f);
    if (f) {
      const int32_t pos = w + __popcll(bm & ((1ull << lane) - 1ull));
      ocol[base + pos] = lo + c;
      oval[base + pos] = acc[c];
    }
    w += __popcll(bm);
  }
  if (lane == 0) ucnt[i] = prior + w;
}

// Inclusive prefix maximum over the wavefront's lanes: row shifts by 1, 2, 4 and 8 within
// each 16-lane row (lanes shifted in from outside the row read -1), then the last lane of
// row 0 (of row 2) into row 1 (row 3), then the last lane of row 1 into rows 2 and 3.
__device__ __forceinline__ int32_t wave_prefix_max(int32_t x) {
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xF, 0xF, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xF, 0xF, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xF, 0xF, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xF, 0xF, false));  // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return x;
}

// ---- rank accumulator (257..1024 products, narrow output rows) -----------------------------
// One wavefront per row.  The row's products are staged in LDS at their Gustavson positions
// (consecutive products on consecutive lanes: each its Y entry's column and X_ik Y_kj, the
// loads of several 64-product steps in flight together), the distinct columns marked in
// a bitmap over the row's column window, and each X entry's products then added, in X order,
// into an accumulator indexed by the column's rank among the row's distinct columns: the
// columns of one Y row are distinct, so the adds of one X entry never collide, and the X
// entries follow each other in the wavefront's program order, so every output entry receives
// its products in ascending k, from 0, as in the sort-based bins.  Rows outside the stage's
// limits are listed in rov for the sort-based kernel of their bin.
constexpr int32_t kRankT = 1024;    // products
constexpr int32_t kRankX = 64;      // X entries (the adds take one step per X entry)
constexpr int32_t kRankW = 65536;   // column window
constexpr int32_t kRankD = 256;     // distinct columns
constexpr int kRankSteps = 8;       // 64-product steps whose loads are issued together
static_assert(kRankX <= 64, "one X entry per lane while staging");
__global__ __launch_bounds__(64) void k_esc_rank(const int32_t *rows, int32_t nrows,
                                                 const int32_t *xrp, const int32_t *xcol,
                                                 const double *xval, const int32_t *xpref,
                                                 const int32_t *yrp, const int32_t *ycol,
                                                 const double *yval, const int64_t *poff,
                                                 int32_t *ocol, double *oval, int32_t *ucnt,
                                                 int32_t *rov, int32_t *nrov) {
  __shared__ int32_t s_c[kRankT];       // staged columns, then their ranks
  __shared__ double s_v[kRankT];        // staged products
  __shared__ uint32_t s_bits[kRankW / 32];
  __shared__ uint16_t s_pre[kRankW / 32];  // set bits in the words before
  __shared__ double s_acc[kRankD];
  __shared__ int32_t s_xo[kRankX + 1];  // X entries' first positions, then T
  __shared__ int32_t s_yb[kRankX], s_mark[64];
  __shared__ double s_xv[kRankX];
  const int lane = threadIdx.x;
  const int32_t slot = blockIdx.x;
  if (slot >= nrows) return;  // block-uniform
  const int32_t i = rows[slot];
  const int64_t base = poff[i];
  const int32_t T = (int32_t)(poff[i + 1] - base);
  const int32_t xb = xrp[i], nx = xrp[i + 1] - xb;
  auto overflow = [&]() {
    if (lane == 0) rov[atomicAdd(nrov, 1)] = i;
  };
  if (nx > kRankX || T > kRankT || T == 0) {  // wavefront-uniform
    overflow();
    return;
  }
  // stage the X entries (lane e holds entry e), then the products in Gustavson order, lane l
  // taking products l, l + 64, ...: product p belongs to the last entry that starts at or
  // before it (among entries with products).  Per 64-product step, each entry starting
  // inside the step marks its first product's lane and a prefix maximum over the lanes, from
  // the entry of the step's preceding product, gives every lane its entry.  kRankSteps steps'
  // entries are found first, then their loads issued together, then their products staged.
  int32_t my_o = 0, my_len = 0;
  if (lane < nx) {
    const int32_t k = xcol[xb + lane];
    my_o = xpref[xb + lane];
    const int32_t yb = yrp[k];
    my_len = yrp[k + 1] - yb;
    s_xo[lane] = my_o;
    s_yb[lane] = yb;
    s_xv[lane] = xval[xb + lane];
  }
  if (lane == 0) s_xo[nx] = T;
  s_mark[lane] = -1;
  __syncthreads();
  const bool starts = lane < nx && my_len > 0;
  int32_t lo = INT_MAX, hi = -1, carry = -1;
  for (int32_t g0 = 0; g0 < T; g0 += 64 * kRankSteps) {
    int32_t ed[kRankSteps], qd[kRankSteps];
#pragma unroll
    for (int d = 0; d < kRankSteps; ++d) {
      const int32_t p0 = g0 + 64 * d;
      ed[d] = 0;
      qd[d] = 0;  // lanes past T load Y's first entry and discard it (T > 0: Y has entries)
      if (p0 < T) {  // wavefront-uniform
        if (starts && my_o >= p0 && my_o < p0 + 64) s_mark[my_o - p0] = lane;
        __syncthreads();
        int32_t e = s_mark[lane];
        s_mark[lane] = -1;  // every slot is -1 again for the next step
        e = max(wave_prefix_max(e), carry);
        carry = __builtin_amdgcn_readlane(e, 63);
        const int32_t p = p0 + lane;
        if (p < T) {
          ed[d] = e;
          qd[d] = s_yb[e] + p - s_xo[e];
        }
      }
    }
    int32_t cd[kRankSteps];
    double vd[kRankSteps];
#pragma unroll
    for (int d = 0; d < kRankSteps; ++d) {
      cd[d] = ycol[qd[d]];
      vd[d] = yval[qd[d]];
    }
#pragma unroll
    for (int d = 0; d < kRankSteps; ++d) {
      const int32_t p = g0 + 64 * d + lane;
      if (p < T) {
        s_c[p] = cd[d];
        s_v[p] = s_xv[ed[d]] * vd[d];
        lo = min(lo, cd[d]);
        hi = max(hi, cd[d]);
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  const int32_t W = hi - lo + 1;
  if (W > kRankW) {  // wavefront-uniform; nothing written to global memory yet
    overflow();
    return;
  }
  const int32_t nw = (W + 31) >> 5;
  for (int32_t w = lane; w < nw; w += 64) s_bits[w] = 0u;
  __syncthreads();
  for (int32_t p = lane; p < T; p += 64) {
    const int32_t c = s_c[p] - lo;
    atomicOr(&s_bits[c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  // popcount prefix over the words: lane l takes a contiguous run of them
  const int32_t wl = (nw + 63) >> 6;
  const int32_t w0 = min(nw, lane * wl), w1 = min(nw, w0 + wl);
  int32_t cnt = 0;
  for (int32_t w = w0; w < w1; ++w) cnt += __popc(s_bits[w]);
  int32_t incl = cnt;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  const int32_t D = __shfl(incl, 63, 64);
  if (D > kRankD) {  // wavefront-uniform
    overflow();
    return;
  }
  int32_t run = incl - cnt;
  for (int32_t w = w0; w < w1; ++w) {
    s_pre[w] = (uint16_t)run;
    run += __popc(s_bits[w]);
  }
  for (int32_t r = lane; r < D; r += 64) s_acc[r] = 0.0;
  __syncthreads();
  // ranks (each position's own lane reads and overwrites it); the columns go out at theirs
  for (int32_t p = lane; p < T; p += 64) {
    const int32_t c = s_c[p] - lo;
    const int32_t w = c >> 5;
    const int32_t r = (int32_t)s_pre[w] + __popc(s_bits[w] & ((1u << (c & 31)) - 1u));
    s_c[p] = r;
    ocol[base + r] = c + lo;  // every position of a column writes the same value
  }
  __syncthreads();
  // the X entries in order; within one, each lane adds its product to its column's sum
  for (int32_t e = 0; e < nx; ++e) {
    const int32_t o0 = s_xo[e], o1 = s_xo[e + 1];
    for (int32_t j = o0 + lane; j < o1; j += 64) {
      const int32_t r = s_c[j];
      s_acc[r] = s_acc[r] + s_v[j];
    }
  }
  __syncthreads();
  for (int32_t r = lane; r < D; r += 64) oval[base + r] = s_acc[r];
  if (lane == 0) ucnt[i] = D;
}

// ---- wavefront-per-row bins (T > 64) ------------------------------------------------------
// One wavefront (a 64-thread block) per row.  The row's products are taken 64 at a time in
// Gustavson order: its X entries are staged 64 at a time with a wave scan of their Y-row
// lengths, and each lane finds its product's entry by binary search over the scan.  A step's
// 64 products are sorted in registers by (column, lane) -- lane order is product order -- and
// the first lane of each run of equal columns adds the run, in order, to that column's
// accumulator in LDS.  Steps follow each other in product order, so every output entry
// receives its products in ascending k, from 0.
//   DENSE  the accumulator is the row's column window (values and a touched bitmap), read
//          out in column order with ballots; rows wider than the LDS (those that overflow the
//          hash bin) are taken in column tiles, one launch per tile, each appending its
//          entries to the row's earlier ones;
//   HASH   an open-addressing table of H slots (every column claimed by an LDS compare-and-
//          swap, its sum starting from 0); a row whose distinct columns pass H/2 is listed in
//          ovf[] to be redone (LDS column tiles, or k_esc_dense).  At the end the occupied
//          slots are compacted and sorted by column (bitonic, in LDS).
// Value of lane (lane ^ J) of the wavefront.  J = 1, 2: a quad permutation (DPP); J = 4, 8:
// the row shifts by J toward the lower lanes (row_shl, lane i reads i + J) and the higher
// lanes (row_shr, lane i reads i - J), of which each lane keeps the one inside its J-group
// pair (both stay inside the 16-lane row); J = 16, 32: an LDS permute.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int lane) {
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  } else if constexpr (J == 4 || J == 8) {
    const uint32_t from_up =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x100 + J, 0xF, 0xF, false);  // row_shl
    const uint32_t from_dn =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x110 + J, 0xF, 0xF, false);  // row_shr
    return (lane & J) ? from_dn : from_up;
  } else {
    return (uint32_t)__shfl_xor((int)v, J, 64);
  }
}
template <int J>
__device__ __forceinline__ uint64_t xor_lane(uint64_t v, int lane) {
  const uint32_t lo = xor_lane<J>((uint32_t)v, lane);
  const uint32_t hi = xor_lane<J>((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
// Ascending bitonic sort of one key per lane across the wavefront (keys distinct).  Keys are
// (column << 6 | lane): 32 bits while the columns stay below 2^26 (one cross-lane move per
// stage), else 64.  Merge K's stage J pairs lanes i and i ^ J.
template <int K, int J, typename KT>
__device__ __forceinline__ KT bitonic_merge(KT key, int lane) {
  const KT other = xor_lane<J>(key, lane);
  const bool up = (lane & K) == 0;
  const bool lower = (lane & J) == 0;
  key = (lower == up) ? (key < other ? key : other) : (key > other ? key : other);
  if constexpr (J > 1)
    return bitonic_merge<K, J / 2>(key, lane);
  else
    return key;
}
template <typename KT, int K = 2>
__device__ __forceinline__ KT wave_sort(KT key, int lane) {
  key = bitonic_merge<K, K / 2>(key, lane);
  if constexpr (K < 64)
    return wave_sort<KT, K * 2>(key, lane);
  else
    return key;
}

template <bool DENSE, int H, typename KT>
__global__ __launch_bounds__(64) void k_esc_wave(
    const int32_t *rows, int32_t nrows, const int32_t *xrp, const int32_t *xcol,
    const double *xval, const int32_t *yrp, const int32_t *ycol, const double *yval,
    int32_t width, const int2 *win, const int64_t *poff, int32_t *ocol, double *oval,
    int32_t *ucnt, int32_t *ovf, int32_t *novf, const int32_t *dcount, int32_t tile,
    int32_t tw) {
  extern __shared__ double lds_dyn[];
  __shared__ int32_t s_incl[64], s_ys[64], s_mark[64];
  __shared__ double s_a[64], s_v[64];
  __shared__ int32_t s_cnt;
  const int lane = threadIdx.x;
  s_mark[lane] = -1;
  const int32_t slot = blockIdx.x;
  if (slot >= (dcount ? *dcount : nrows)) return;  // block-uniform
  const int32_t i = rows[slot];
  const int64_t base = poff[i];
  // DENSE: acc[width] then the bitmap; HASH: hv[H], hk[H], then the sort keys (H/2)
  double *acc = lds_dyn;
  uint32_t *bits = reinterpret_cast<uint32_t *>(acc + width);
  double *hv = lds_dyn;
  int32_t *hk = reinterpret_cast<int32_t *>(hv + H);
  uint64_t *sk = reinterpret_cast<uint64_t *>(hk + H);
  int32_t lo = 0, rw = width, prior = 0;
  if (DENSE) {
    if (win) {
      const int2 w = win[slot];
      lo = w.x;
      rw = w.y;
    }
    if (tw > 0) {  // column tile `tile` of the window, appended to the earlier tiles' entries
      const int32_t off = tile * tw;
      if (tile > 0 && off >= rw) return;  // block-uniform: the row's window ended earlier
      lo += off;
      rw = min(tw, rw - off);
      if (tile > 0) prior = ucnt[i];
    }
    for (int32_t c = lane; c < rw; c += 64) acc[c] = 0.0;
    for (int32_t c = lane; c < ((rw + 31) >> 5); c += 64) bits[c] = 0u;
  } else {
    for (int32_t c = lane; c < H; c += 64) {
      hk[c] = -1;
      hv[c] = 0.0;
    }
    if (lane == 0) s_cnt = 0;
  }
  __syncthreads();
  bool over = false;  // block-uniform
  const int32_t xb = xrp[i], xe = xrp[i + 1];
  for (int32_t e0 = xb; e0 < xe && !over; e0 += 64) {
    const int32_t cnt = min(64, xe - e0);
    int32_t len = 0, ys = 0;
    double a = 0.0;
    if (lane < cnt) {
      const int32_t k = xcol[e0 + lane];
      a = xval[e0 + lane];
      ys = yrp[k];
      len = yrp[k + 1] - ys;
    }
    int32_t incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    const int32_t tot = __shfl(incl, 63, 64);
    __syncthreads();  // the previous chunk's searches are done
    s_incl[lane] = incl;
    s_ys[lane] = ys;
    s_a[lane] = a;
    __syncthreads();
    // product p of the chunk belongs to the last staged entry g that starts at or before it
    // (among entries with products), at offset p - s_incl[g-1] in its row of Y.  For a step
    // of 64 products, each entry starting inside the step marks its first product's lane, and
    // a prefix maximum over the lanes, from the entry of the step's preceding product, gives
    // every lane its entry.  The next step's entry is loaded before this step is sorted and
    // added, so its latency overlaps them (the product is formed when it is used).
    const int32_t ex = incl - len;  // this lane's entry's first product
    const bool starts = lane < cnt && len > 0;
    int32_t carry = -1;  // entry of the product before the step being fetched (wave-uniform)
    int32_t jn = -1;
    double yn = 0.0, an = 0.0;
    auto fetch = [&](int32_t p0) {
      jn = -1;
      if (p0 >= tot) return;  // wave-uniform
      if (starts && ex >= p0 && ex < p0 + 64) s_mark[ex - p0] = lane;
      __syncthreads();
      int32_t g = s_mark[lane];
      s_mark[lane] = -1;  // every slot is -1 again for the next step
      g = max(wave_prefix_max(g), carry);
      carry = __builtin_amdgcn_readlane(g, 63);
      const int32_t p = p0 + lane;
      if (p < tot) {
        const int32_t q = s_ys[g] + p - (g > 0 ? s_incl[g - 1] : 0);
        jn = ycol[q];
        yn = yval[q];
        an = s_a[g];
      }
    };
    fetch(0);
    for (int32_t p0 = 0; p0 < tot; p0 += 64) {
      const int32_t j = jn;
      const double y = yn, a = an;
      fetch(p0 + 64);
      constexpr KT kNone = ~KT(0);
      KT key = kNone;
      double v = 0.0;
      if (j >= 0) {
        v = a * y;
        key = ((KT)(uint32_t)j << 6) | (KT)lane;
      }
      key = wave_sort<KT>(key, lane);
      const double sv = __shfl(v, (int)(key & 63u), 64);
      const int32_t col = key == kNone ? -1 : (int32_t)(key >> 6);
      // runs of equal columns: a run starts where the column differs from the lane below;
      // it ends at the next start or at the last product (empty keys sort last)
      const int32_t below = __shfl_up(col, 1, 64);
      const bool head = col >= 0 && (lane == 0 || below != col);
      const uint64_t heads = __ballot(head);
      const int32_t nprod = __popcll(__ballot(col >= 0));
      const uint64_t later = lane < 63 ? heads >> (lane + 1) : 0ull;
      const int32_t end = later ? lane + 1 + (int32_t)__builtin_ctzll(later) : nprod;
      s_v[lane] = sv;
      __syncthreads();
      if (head) {
        if (DENSE) {
          const int32_t c = col - lo;  // outside the window only with tiles
          if ((uint32_t)c < (uint32_t)rw) {
            double t = acc[c];
            for (int r = lane; r < end; ++r) t += s_v[r];
            acc[c] = t;
            atomicOr(&bits[c >> 5], 1u << (c & 31));
          }
        } else {
          uint32_t h = hash_slot(col, H - 1);
          for (int probe = 0; probe < H; ++probe) {
            const int32_t old = atomicCAS(&hk[h], -1, col);
            if (old == -1) {
              atomicAdd(&s_cnt, 1);
              break;
            }
            if (old == col) break;
            h = (h + 1) & (H - 1);
          }
          double t = hv[h];
          for (int r = lane; r < end; ++r) t += s_v[r];
          hv[h] = t;
        }
      }
      __syncthreads();
      if (!DENSE && 2 * s_cnt > H) {  // block-uniform: too many columns for the table
        over = true;
        break;
      }
    }
  }
  if (over) {
    if (lane == 0) ovf[atomicAdd(novf, 1)] = i;
    return;
  }
  if (DENSE) {
    int32_t w = 0;
    for (int32_t c0 = 0; c0 < rw; c0 += 64) {
      const int32_t c = c0 + lane;
      const bool f = c < rw && ((bits[c >> 5] >> (c & 31)) & 1u);
      const unsigned long long bm = __ballot(f);
      if (f) {
        const int32_t pos = w + __popcll(bm & ((1ull << lane) - 1ull));
        ocol[base + prior + pos] = lo + c;
        oval[base + prior + pos] = acc[c];
      }
      w += __popcll(bm);
    }
    if (lane == 0) ucnt[i] = prior + w;
  } else {
    // compact the occupied slots as (column << 32 | slot) keys, sort them, write in order
    int32_t u = 0;
    for (int32_t c0 = 0; c0 < H; c0 += 64) {
      const int32_t c = c0 + lane;
      const int32_t kc = hk[c];
      const bool f = kc >= 0;
      const unsigned long long bm = __ballot(f);
      if (f)
        sk[u + __popcll(bm & ((1ull << lane) - 1ull))] =
            ((uint64_t)(uint32_t)kc << 32) | (uint32_t)c;
      u += __popcll(bm);
    }
    int32_t up = 1;
    while (up < u) up <<= 1;
    for (int32_t q = u + lane; q < up; q += 64) sk[q] = ~0ull;
    __syncthreads();
    for (int32_t kk = 2; kk <= up; kk <<= 1) {
      for (int32_t j = kk >> 1; j > 0; j >>= 1) {
        for (int32_t idx = lane; idx < up; idx += 64) {
          const int32_t ixj = idx ^ j;
          if (ixj > idx) {
            const uint64_t x = sk[idx], y = sk[ixj];
            if ((x > y) == ((idx & kk) == 0)) {
              sk[idx] = y;
              sk[ixj] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int32_t r = lane; r < u; r += 64) {
      ocol[base + r] = (int32_t)(sk[r] >> 32);
      oval[base + r] = hv[(uint32_t)sk[r]];
    }
    if (lane == 0) ucnt[i] = u;
  }
}

// Largest output width the LDS bin takes on this device: the opt-in LDS per workgroup less
// the kernel's static LDS, at 8 bytes plus one bit per column (queried once per device).
static int32_t lds_cols_max() {
  static std::mutex mu;
  static int32_t cache[64];
  static bool done[64];
  int dev = 0;
  SA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lock(mu);
  if (!done[dev]) {
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) !=
            hipSuccess ||
        optin <= 0)
      optin = 64 << 10;
    const int64_t avail = (int64_t)optin - 4096;  // the kernel's static LDS is under 2 KB
    int32_t cols = (int32_t)((avail * 8) / 65);     // 8 bytes + 1 bit per column
    cols &= ~31;
    const int bytes = (int)(((int64_t)cols * 65 + 7) / 8);
    if (cols > (64 << 10) / 9 &&
        (hipFuncSetAttribute((const void *)k_esc_wave<true, 1, uint32_t>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess ||
         hipFuncSetAttribute((const void *)k_esc_wave<true, 1, uint64_t>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess ||
         hipFuncSetAttribute((const void *)k_esc_lds<kLdsDepth>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess))
      cols = (((64 << 10) - 4096) * 8 / 65) & ~31;
    cache[dev] = cols;
    done[dev] = true;
  }
  return cache[dev];
}

// Short rows: a wavefront takes 64 consecutive rows, whose entries are one contiguous run of
// C.  At most 16 entries per row on average: lanes copy consecutive entries (coalesced
// writes), each finding its row by binary search over the 64 row starts held in LDS; more:
// row by row, 64 lanes per row (both sides contiguous).
__global__ __launch_bounds__(kBlock) void k_compact_w(int32_t m, const int64_t *poff,
                                                      const int32_t *crp, const int32_t *ocol,
                                                      const double *oval, int32_t *ccol,
                                                      double *cval) {
  constexpr int NW = kBlock / 64;
  __shared__ int32_t s_rp[NW][65];
  __shared__ int64_t s_po[NW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * NW + w) * 64;  // this wavefront's first row
  const int64_t row = r0 + lane;
  s_rp[w][lane] = crp[row < m ? row : m];  // rows past the end: empty, at C's end
  if (lane == 0) s_rp[w][64] = crp[r0 + 64 < m ? r0 + 64 : m];
  s_po[w][lane] = row < m ? poff[row] : 0;
  __syncthreads();
  const int32_t d0 = s_rp[w][0], d1 = s_rp[w][64];
  if (d1 - d0 <= 64 * 16) {  // wave-uniform: short rows, one search per entry
    for (int32_t d = d0 + lane; d < d1; d += 64) {
      int32_t lo = 0, hi = 63;  // last row r with s_rp[r] <= d (empty rows share starts)
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_rp[w][mid] <= d) lo = mid;
        else hi = mid - 1;
      }
      const int64_t src = s_po[w][lo] + (d - s_rp[w][lo]);
      ccol[d] = ocol[src];
      cval[d] = oval[src];
    }
  } else {  // longer rows: row by row, 64 lanes per row
    for (int r = 0; r < 64; ++r) {
      const int32_t rb = s_rp[w][r], re = s_rp[w][r + 1];
      const int64_t shift = s_po[w][r] - rb;
      for (int32_t d = rb + lane; d < re; d += 64) {
        ccol[d] = ocol[shift + d];
        cval[d] = oval[shift + d];
      }
    }
  }
}

// One thread per output entry: find the entry's row by binary search over C's row pointers
// and copy from the row's slot area (coalesced writes; long rows).
__global__ void k_compact(int32_t m, int64_t nnz, const int64_t *poff, const int32_t *crp,
                          const int32_t *ocol, const double *oval, int32_t *ccol, double *cval) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int32_t lo = 0, hi = m - 1;  // last row with crp[row] <= e
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if ((int64_t)crp[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  const int64_t src = poff[lo] + (e - crp[lo]);
  ccol[e] = ocol[src];
  cval[e] = oval[src];
}

__global__ void k_put_total(const int64_t *src, int64_t *dst) { *dst = *src; }

// Bins the rows counted by k_count_products_w (one block per row there).
__global__ __launch_bounds__(kBlock) void k_bin_rows(int32_t m, const int64_t *poff,
                                                     int32_t *lists, int32_t *counters) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i64 < m;
  const int32_t i = live ? (int32_t)i64 : 0;
  bin_row(live, i, live ? poff[i + 1] - poff[i] : 0, m, lists, counters);
}

// Column tiles that the hash bin's overflowing rows may take in LDS (environment variable
// SAAMG_SPGEMM_MAX_TILES; 0 sends them to the dense accumulator in global memory).
static int32_t max_tiles() {
  const char *e = std::getenv("SAAMG_SPGEMM_MAX_TILES");
  return e ? std::atoi(e) : 8;
}

// k_esc_wave with 32-bit sort keys when every column of Y fits in 26 bits, else 64-bit keys
// (the environment variable SAAMG_SPGEMM_KEY64=1 takes the 64-bit keys at any width).
template <bool DENSE, int H, typename... Args>
void launch_esc_wave(int32_t ncols, unsigned grid, size_t lds, hipStream_t s, Args... args) {
  const char *e = std::getenv("SAAMG_SPGEMM_KEY64");
  const bool key64 = e && std::atoi(e) != 0;
  if (ncols < (1 << 26) && !key64)
    k_esc_wave<DENSE, H, uint32_t><<<grid, 64, lds, s>>>(args...);
  else
    k_esc_wave<DENSE, H, uint64_t><<<grid, 64, lds, s>>>(args...);
}

void spgemm(const Csr &X, const Csr &Y, Arena &ar, Csr &C, hipStream_t s) {
  const int32_t m = X.n;
  C.n = m;
  C.ncols = Y.ncols;
  C.maxrow = -1;
  Arena tmp;
  tmp.stream = s;
  int64_t *cnt = tmp.alloc<int64_t>(m + 1);
  int32_t *xpref = tmp.alloc<int32_t>(X.nnz > 0 ? X.nnz : 1);
  int64_t *poff = tmp.alloc<int64_t>(m + 1);
  int32_t *lists = tmp.alloc<int32_t>(kBins * (int64_t)(m > 0 ? m : 1));
  // kBins bin sizes, the overflow count, the widest row window, then the product total (64
  // bits)
  int32_t *counters = tmp.alloc<int32_t>(10);
  fill_i32(counters, 0, 8, s);
  // rows of up to 64 entries: a thread per row, which also bins the row; longer: a
  // wavefront per row, binned after the scan
  const bool wave_count =
      m > 0 && (X.maxrow >= 0 ? X.maxrow : max_row_length(m, X.rp, s)) > 64;
  if (wave_count)
    k_count_products_w<<<(unsigned)m, 64, 0, s>>>(m, X.rp, X.col, Y.rp, cnt, xpref);
  else if (m > 0)
    k_count_products<<<grid_for(m), kBlock, 0, s>>>(m, X.rp, X.col, Y.rp, cnt, xpref, lists,
                                                    counters);
  SA_LAUNCH_CHECK();
  exclusive_scan_i64(cnt, poff, m, s);
  if (wave_count) {
    k_bin_rows<<<grid_for(m), kBlock, 0, s>>>(m, poff, lists, counters);
    SA_LAUNCH_CHECK();
  }
  // the bin sizes and the product total in one readback
  k_put_total<<<1, 1, 0, s>>>(poff + m, (int64_t *)(counters + 8));
  SA_LAUNCH_CHECK();
  int32_t hc[10];
  readback(hc, counters, sizeof(hc), s);
  int64_t total = 0;
  std::memcpy(&total, hc + 8, sizeof(total));
  int32_t *ocol = tmp.alloc<int32_t>(total > 0 ? total : 1);
  double *oval = tmp.alloc<double>(total > 0 ? total : 1);
  int32_t *ucnt = tmp.alloc<int32_t>(m + 1);
  const int32_t *lg[3] = {lists, lists + m, lists + 2 * (int64_t)m};
  const int32_t *l1 = lists + 3 * (int64_t)m, *l2 = lists + 4 * (int64_t)m,
                *l3 = lists + 5 * (int64_t)m;
  // two products per lane: 8, 4 and 2 rows per wavefront for the <= 16, <= 32, <= 64 bins
  if (hc[0] > 0)
    k_esc_group<8, 2><<<(unsigned)ceil_div(hc[0], kWave / 8), kWave, 0, s>>>(
        lg[0], hc[0], X.rp, X.col, X.val, Y.rp, Y.col, Y.val, poff, ocol, oval, ucnt);
  if (hc[1] > 0)
    k_esc_group<16, 2><<<(unsigned)ceil_div(hc[1], kWave / 16), kWave, 0, s>>>(
        lg[1], hc[1], X.rp, X.col, X.val, Y.rp, Y.col, Y.val, poff, ocol, oval, ucnt);
  if (hc[2] > 0)
    k_esc_group<32, 2><<<(unsigned)ceil_div(hc[2], kWave / 32), kWave, 0, s>>>(
        lg[2], hc[2], X.rp, X.col, X.val, Y.rp, Y.col, Y.val, poff, ocol, oval, ucnt);
  SA_LAUNCH_CHECK();
  const int32_t n256 = hc[3], n1024 = hc[4], nlong = hc[5];  // wavefront-per-row bins
  int32_t *ovf = nullptr;
  if (n256 > 0 || n1024 > 0 || nlong > 0) ovf = tmp.alloc<int32_t>(n256 + n1024 + nlong);
  // T <= 256: the wavefront kernel with a 512-slot hash table (at least 2T slots: it never
  // overflows); T <= 1024: one block per row, the whole row sorted in LDS.  With Y rows of 8
  // entries or more on average (R (AP)), the rank-accumulator kernel takes the rows of the
  // second bin first and leaves those outside its limits to the block sort (their count read
  // on the device).
  const bool rank = Y.nnz >= 8 * (int64_t)Y.n && n1024 > 0;
  const int32_t *r1024 = l2, *c1024 = nullptr;
  if (rank) {
    int32_t *rov = tmp.alloc<int32_t>(n1024);
    int32_t *rc = tmp.alloc<int32_t>(1);
    fill_i32(rc, 0, 1, s);
    k_esc_rank<<<(unsigned)n1024, 64, 0, s>>>(l2, n1024, X.rp, X.col, X.val, xpref, Y.rp, Y.col,
                                              Y.val, poff, ocol, oval, ucnt, rov, rc);
    SA_LAUNCH_CHECK();
    r1024 = rov;
    c1024 = rc;
  }
  if (n256 > 0) {
    launch_esc_wave<false, 512>(Y.ncols, (unsigned)n256, 16 * 512, s, l1, n256, X.rp, X.col,
                                X.val, Y.rp, Y.col, Y.val, 0, nullptr, poff, ocol, oval, ucnt,
                                ovf, counters + kBins, nullptr, 0, 0);
    SA_LAUNCH_CHECK();
  }
  if (n1024 > 0) {
    k_esc_single<256><<<(unsigned)n1024, 256, 0, s>>>(r1024, n1024, X.rp, X.col, X.val, xpref,
                                                      Y.rp, Y.col, Y.val, poff, ocol, oval,
                                                      ucnt, c1024);
    SA_LAUNCH_CHECK();
  }
  // long rows: the dense window accumulator when Y's width fits the LDS (sized to the widest
  // row window; up to 2048 columns the whole width), else a 2048-slot hash table whose
  // overflowing rows (more than 1024 distinct columns) are redone below
  const bool lds_bin = Y.ncols <= lds_cols_max();
  int32_t wmax = Y.ncols;
  int2 *win = nullptr;
  if (nlong > 0 && lds_bin && Y.ncols > 2048) {
    win = tmp.alloc<int2>(nlong);
    fill_i32(counters + kBins + 1, 0, 1, s);
    k_row_window<<<grid_for((int64_t)nlong * 64), kBlock, 0, s>>>(l3, nlong, X.rp, X.col, Y.rp,
                                                                  Y.col, win,
                                                                  counters + kBins + 1);
    SA_LAUNCH_CHECK();
    wmax = read1(counters + kBins + 1, s);
  }
  if (nlong > 0 && lds_bin) {
    const int32_t wl = (wmax + 31) & ~31;
    const size_t lds = (size_t)wl * sizeof(double) + (size_t)(wl / 32) * 4;
    // Y rows of 16 entries or more on average (R (AP)): one X entry per step, its Y row
    // across the lanes; shorter Y rows (A P): 64 products per step, sorted
    if (Y.nnz >= 16 * (int64_t)Y.n)
      k_esc_lds<kLdsDepth><<<(unsigned)nlong, 64, lds, s>>>(l3, nlong, X.rp, X.col, X.val, Y.rp,
                                                           Y.col, Y.val, wl, win, poff, ocol,
                                                           oval, ucnt, 0, 0);
    else
      launch_esc_wave<true, 1>(Y.ncols, (unsigned)nlong, lds, s, l3, nlong, X.rp, X.col, X.val,
                               Y.rp, Y.col, Y.val, wl, win, poff, ocol, oval, ucnt, ovf,
                               counters + kBins, nullptr, 0, 0);
    SA_LAUNCH_CHECK();
  } else if (nlong > 0) {
    launch_esc_wave<false, 2048>(Y.ncols, (unsigned)nlong, 16 * 2048, s, l3, nlong, X.rp,
                                 X.col, X.val, Y.rp, Y.col, Y.val, 0, nullptr, poff, ocol, oval,
                                 ucnt, ovf, counters + kBins, nullptr, 0, 0);
    SA_LAUNCH_CHECK();
    const int32_t nov = read1(counters + kBins, s);
    // rows over 1024 distinct columns: their column windows in LDS tiles (one launch per tile,
    // at most kMaxTiles), else a dense accumulator in global memory
    int32_t ntile = 0, tw = 0;
    int2 *owin = nullptr;
    if (nov > 0) {
      owin = tmp.alloc<int2>(nov);
      fill_i32(counters + kBins + 1, 0, 1, s);
      k_row_window<<<grid_for((int64_t)nov * 64), kBlock, 0, s>>>(ovf, nov, X.rp, X.col, Y.rp,
                                                                 Y.col, owin,
                                                                 counters + kBins + 1);
      SA_LAUNCH_CHECK();
      const int32_t wmax = read1(counters + kBins + 1, s);
      tw = std::min(lds_cols_max(), (wmax + 31) & ~31);
      ntile = tw > 0 ? (int32_t)ceil_div(wmax, tw) : 0;
      if (ntile > max_tiles()) ntile = 0;
    }
    if (ntile > 0) {
      const size_t lds = (size_t)tw * sizeof(double) + (size_t)(tw / 32) * 4;
      for (int32_t t = 0; t < ntile; ++t) {
        if (Y.nnz >= 16 * (int64_t)Y.n)
          k_esc_lds<kLdsDepth><<<(unsigned)nov, 64, lds, s>>>(ovf, nov, X.rp, X.col, X.val,
                                                             Y.rp, Y.col, Y.val, tw, owin, poff,
                                                             ocol, oval, ucnt, t, tw);
        else
          launch_esc_wave<true, 1>(Y.ncols, (unsigned)nov, lds, s, ovf, nov, X.rp, X.col, X.val,
                                   Y.rp, Y.col, Y.val, tw, owin, poff, ocol, oval, ucnt,
                                   nullptr, nullptr, nullptr, t, tw);
        SA_LAUNCH_CHECK();
      }
    } else if (nov > 0) {
      // dense accumulators: at most ~2 GiB of them at once
      const int64_t per = (int64_t)Y.ncols * 12;
      int64_t nb = std::min<int64_t>(nov, std::max<int64_t>(1, (int64_t(2) << 30) / per));
      nb = std::min<int64_t>(nb, 1024);
      double *dacc = tmp.alloc<double>(nb * (int64_t)Y.ncols);
      int32_t *dflag = tmp.alloc<int32_t>(nb * (int64_t)Y.ncols);
      k_esc_dense<<<(unsigned)nb, kBlock, 0, s>>>(ovf, nov, X.rp, X.col, X.val, xpref, Y.rp,
                                                  Y.col, Y.val, Y.ncols, poff, ocol, oval, ucnt,
                                                  dacc, dflag);
      SA_LAUNCH_CHECK();
    }
  }
  C.rp = ar.alloc<int32_t>(m + 1);
  exclusive_scan_i32(ucnt, C.rp, m, s);
  C.nnz = read1(C.rp + m, s);
  C.col = ar.alloc<int32_t>(C.nnz);
  C.val = ar.alloc<double>(C.nnz);
  if (C.nnz > 0) {
    if (C.nnz <= 20 * (int64_t)m)  // short rows on average: wavefronts over 64 rows
      k_compact_w<<<(unsigned)ceil_div(m, kBlock), kBlock, 0, s>>>(m, poff, C.rp, ocol, oval,
                                                                 C.col, C.val);
    else
      k_compact<<<grid_for(C.nnz), kBlock, 0, s>>>(m, C.nnz, poff, C.rp, ocol, oval, C.col,
                                                   C.val);
    SA_LAUNCH_CHECK();
  }
}

// ---- numeric plan for a fixed pattern (re-setup) ---------------------------------------------
// Built once from the patterns of X, Y and C, in parallel over X's entries (a thread per
// entry, or a wavefront per entry when Y's rows are long): every product (e, q) finds its
// column in C's sorted row i by binary search.  Pass 1 counts the products of every C entry
// (atomically), pass 2 lists them in arrival order, and a last pass sorts every list by X
// position e, i.e. by inner index: within one list each e occurs once, so the order is total.
__device__ inline int32_t plan_find(const int32_t *ccol, int32_t lo, int32_t hi, int32_t j) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (ccol[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
__global__ void k_entry_rows(int32_t m, const int32_t *rp, int32_t *row) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= m) return;
  const int32_t i = (int32_t)i64;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) row[e] = i;
}
// G lanes per X entry (1 or 64); FILL: place (e, q) at lrp[p] + the next free slot of p.
template <int G, bool FILL>
__global__ void k_plan_entries(int64_t nx, const int32_t *__restrict__ xrow,
                               const int32_t *__restrict__ xcol, const int32_t *__restrict__ yrp,
                               const int32_t *__restrict__ ycol,
                               const int32_t *__restrict__ crp,
                               const int32_t *__restrict__ ccol, int32_t *cnt,
                               const int64_t *__restrict__ lrp, int32_t *le, int32_t *lq,
                               int32_t *err, int32_t bit) {
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int32_t lane = G == 1 ? 0 : (int32_t)(threadIdx.x % G);
  if (g >= nx) return;
  const int32_t e = (int32_t)g;
  const int32_t i = xrow[e], k = xcol[e];
  const int32_t cb = crp[i], ce = crp[i + 1];
  for (int32_t q = yrp[k] + lane; q < yrp[k + 1]; q += G) {
    const int32_t j = ycol[q];
    const int32_t p = plan_find(ccol, cb, ce, j);
    if (p >= ce || ccol[p] != j) {
      atomicOr(err, bit);
      continue;
    }
    const int32_t slot = atomicAdd(cnt + p, 1);
    if (FILL) {
      le[lrp[p] + slot] = e;
      lq[lrp[p] + slot] = q;
    }
  }
}
// Thread per C entry: a list of up to kPlanShort entries sorted by X position in place
// (insertion); longer lists are listed for k_plan_sort_long.
constexpr int32_t kPlanShort = 32;
constexpr int32_t kPlanLds = 4096;  // a list is at most as long as X's longest row
__global__ void k_plan_sort(int32_t nnzc, const int64_t *__restrict__ lrp, int32_t *le,
                            int32_t *lq, int32_t *longs, int32_t *nlong) {
  const int64_t p64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p64 >= nnzc) return;
  const int64_t b = lrp[p64], en = lrp[p64 + 1];
  if (en - b > kPlanShort) {
    longs[atomicAdd(nlong, 1)] = (int32_t)p64;
    return;
  }
  for (int64_t t = b + 1; t < en; ++t) {
    const int32_t ke = le[t], kq = lq[t];
    int64_t u = t - 1;
    while (u >= b && le[u] > ke) {
      le[u + 1] = le[u];
      lq[u + 1] = lq[u];
      --u;
    }
    le[u + 1] = ke;
    lq[u + 1] = kq;
  }
}
// Block per long list (grid-stride over them): keys (e << 32 | q) sorted by a bitonic sort in
// LDS (e is unique within a list, so the order is that of e); a list past kPlanLds entries (X
// rows that long) falls back to thread 0's insertion sort.
__global__ __launch_bounds__(kBlock) void k_plan_sort_long(const int32_t *__restrict__ longs,
                                                           const int32_t *__restrict__ nlong,
                                                           const int64_t *__restrict__ lrp,
                                                           int32_t *le, int32_t *lq) {
  __shared__ uint64_t key[kPlanLds];
  const int32_t nl = *nlong;
  for (int32_t idx = blockIdx.x; idx < nl; idx += gridDim.x) {
    const int32_t p = longs[idx];
    const int64_t b = lrp[p];
    const int32_t len = (int32_t)(lrp[p + 1] - b);
    if (len > kPlanLds) {  // block-uniform
      if (threadIdx.x == 0) {
        for (int32_t t = 1; t < len; ++t) {
          const int32_t ke = le[b + t], kq = lq[b + t];
          int32_t u = t - 1;
          while (u >= 0 && le[b + u] > ke) {
            le[b + u + 1] = le[b + u];
            lq[b + u + 1] = lq[b + u];
            --u;
          }
          le[b + u + 1] = ke;
          lq[b + u + 1] = kq;
        }
      }
      __syncthreads();
      continue;
    }
    int32_t L = 1;
    while (L < len) L <<= 1;
    for (int32_t t = threadIdx.x; t < L; t += blockDim.x)
      key[t] = t < len ? (((uint64_t)(uint32_t)le[b + t] << 32) | (uint32_t)lq[b + t]) : ~0ull;
    __syncthreads();
    for (int32_t kk = 2; kk <= L; kk <<= 1) {
      for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
        for (int32_t t = threadIdx.x; t < L; t += blockDim.x) {
          const int32_t u = t ^ jj;
          if (u > t) {
            const uint64_t x = key[t], y = key[u];
            if ((x > y) == ((t & kk) == 0)) {
              key[t] = y;
              key[u] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int32_t t = threadIdx.x; t < len; t += blockDim.x) {
      le[b + t] = (int32_t)(key[t] >> 32);
      lq[b + t] = (int32_t)(uint32_t)key[t];
    }
    __syncthreads();
  }
}
__global__ void k_plan_numeric(int32_t nnzc, const int64_t *__restrict__ lrp,
                               const int32_t *__restrict__ le, const int32_t *__restrict__ lq,
                               const double *__restrict__ xv, const double *__restrict__ yv,
                               double *__restrict__ cv) {
  const int64_t p64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p64 >= nnzc) return;
  const int32_t p = (int32_t)p64;
  double s = 0.0;
  for (int64_t t = lrp[p]; t < lrp[p + 1]; ++t) s += xv[le[t]] * yv[lq[t]];
  cv[p] = s;
}

__global__ void k_widen_i32(int64_t n, const int32_t *a, int64_t *b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
static void widen_i32(const int32_t *a, int64_t *b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_widen_i32<<<grid_for(n), kBlock, 0, s>>>(n, a, b);
  SA_LAUNCH_CHECK();
}

void spgemm_plan(const Csr &X, const Csr &Y, const Csr &C, Arena &ar, SpgemmPlan &pl,
                 int32_t *err, int32_t bit, hipStream_t s) {
  pl = SpgemmPlan{};
  Arena tmp;
  tmp.stream = s;
  const int64_t nx = X.nnz;
  int32_t *xrow = tmp.alloc<int32_t>(nx > 0 ? nx : 1);
  int32_t *cnt = tmp.alloc<int32_t>(C.nnz + 1);
  pl.lrp = ar.alloc<int64_t>(C.nnz + 1);
  int64_t *cnt64 = tmp.alloc<int64_t>(C.nnz + 1);
  fill_i32(cnt, 0, C.nnz + 1, s);
  if (X.n > 0) {
    k_entry_rows<<<grid_for(X.n), kBlock, 0, s>>>(X.n, X.rp, xrow);
    SA_LAUNCH_CHECK();
  }
  // long Y rows: a wavefront per X entry
  const bool wide = (Y.maxrow >= 0 ? Y.maxrow : max_row_length(Y.n, Y.rp, s)) > 32;
  auto pass = [&](bool fill) {
    if (nx <= 0) return;
    if (wide) {
      if (fill)
        k_plan_entries<64, true><<<grid_for(nx * 64), kBlock, 0, s>>>(
            nx, xrow, X.col, Y.rp, Y.col, C.rp, C.col, cnt, pl.lrp, pl.le, pl.lq, err, bit);
      else
        k_plan_entries<64, false><<<grid_for(nx * 64), kBlock, 0, s>>>(
            nx, xrow, X.col, Y.rp, Y.col, C.rp, C.col, cnt, nullptr, nullptr, nullptr, err,
            bit);
    } else {
      if (fill)
        k_plan_entries<1, true><<<grid_for(nx), kBlock, 0, s>>>(
            nx, xrow, X.col, Y.rp, Y.col, C.rp, C.col, cnt, pl.lrp, pl.le, pl.lq, err, bit);
      else
        k_plan_entries<1, false><<<grid_for(nx), kBlock, 0, s>>>(
            nx, xrow, X.col, Y.rp, Y.col, C.rp, C.col, cnt, nullptr, nullptr, nullptr, err,
            bit);
    }
    SA_LAUNCH_CHECK();
  };
  pass(false);
  widen_i32(cnt, cnt64, C.nnz, s);
  exclusive_scan_i64(cnt64, pl.lrp, C.nnz, s);
  pl.nprod = read1(pl.lrp + C.nnz, s);
  pl.le = ar.alloc<int32_t>(pl.nprod > 0 ? pl.nprod : 1);
  pl.lq = ar.alloc<int32_t>(pl.nprod > 0 ? pl.nprod : 1);
  fill_i32(cnt, 0, C.nnz + 1, s);
  pass(true);
  if (C.nnz > 0) {
    int32_t *longs = tmp.alloc<int32_t>(C.nnz);
    int32_t *nlong = tmp.alloc<int32_t>(1);
    fill_i32(nlong, 0, 1, s);
    k_plan_sort<<<grid_for(C.nnz), kBlock, 0, s>>>((int32_t)C.nnz, pl.lrp, pl.le, pl.lq, longs,
                                                   nlong);
    k_plan_sort_long<<<1024, kBlock, 0, s>>>(longs, nlong, pl.lrp, pl.le, pl.lq);
    SA_LAUNCH_CHECK();
  }
}

void spgemm_numeric(const Csr &X, const Csr &Y, const SpgemmPlan &pl, Csr &C, hipStream_t s) {
  if (C.nnz <= 0) return;
  k_plan_numeric<<<grid_for(C.nnz), kBlock, 0, s>>>((int32_t)C.nnz, pl.lrp, pl.le, pl.lq, X.val,
                                                    Y.val, C.val);
  SA_LAUNCH_CHECK();
}

// R = P^T: entry k of P (row i, column c) sits in R's row c at column i.
__global__ void k_transpose_perm(int32_t n, const int32_t *__restrict__ prp,
                                 const int32_t *__restrict__ pcol,
                                 const int32_t *__restrict__ rrp,
                                 const int32_t *__restrict__ rcol, int32_t *perm) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= n) return;
  const int32_t i = (int32_t)i64;
  for (int32_t k = prp[i]; k < prp[i + 1]; ++k) {
    const int32_t c = pcol[k];
    const int32_t p = plan_find(rcol, rrp[c], rrp[c + 1], i);
    perm[k] = (p < rrp[c + 1] && rcol[p] == i) ? p : -1;  // -1: never, for R = P^T
  }
}
__global__ void k_transpose_values(int64_t nnz, const int32_t *__restrict__ perm,
                                   const double *__restrict__ pv, double *__restrict__ rv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz && perm[k] >= 0) rv[perm[k]] = pv[k];
}
void transpose_perm(const Csr &P, const Csr &R, Arena &ar, int32_t **perm, hipStream_t s) {
  *perm = ar.alloc<int32_t>(P.nnz > 0 ? P.nnz : 1);
  if (P.n > 0) {
    k_transpose_perm<<<grid_for(P.n), kBlock, 0, s>>>(P.n, P.rp, P.col, R.rp, R.col, *perm);
    SA_LAUNCH_CHECK();
  }
}
void transpose_values(const Csr &P, const int32_t *perm, Csr &R, hipStream_t s) {
  if (P.nnz <= 0) return;
  k_transpose_values<<<grid_for(P.nnz), kBlock, 0, s>>>(P.nnz, perm, P.val, R.val);
  SA_LAUNCH_CHECK();
}

}  // namespace sa
