// Setup kernels: CSR validation, strength of connection, the aggregation graph, parallel
// root selection, aggregation, Sprsfy, filtered matrix with its smoothing diagonal, power
// method, prolongator smoothing, Cnstrnt, transpose.
//
// Every floating-point reduction runs in the order the method's definition fixes (row sums
// sequential in ascending column order from 0), with FMA contraction disabled at compile
// time, so the setup is deterministic and equal to the sequential definition bit for bit.
// Setup kernels are one thread per row (rows hold 5-30 entries on the fine levels); they
// run once per level and are bound by HBM traffic or by the level's size.
#include <chrono>
#include <climits>
#include <cstdlib>
#include <type_traits>

#include "kernels.hpp"

namespace sa {

#define SA_ROW_KERNEL_BEGIN(n)                                    \
  const int64_t i64_ = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; \
  if (i64_ >= (n)) return;                                        \
  const int32_t i = (int32_t)i64_;

// ---- one wavefront per row (levels with long rows) ------------------------------------------
// Kernels below with a _w suffix process one row per 64-thread block (one wavefront), lanes
// striding over the row.  Floating-point sums keep the sequential order: terms are staged in
// LDS 64 at a time and lane 0 adds them in ascending entry order from 0.  A term outside the
// summed subset contributes +0.0, which leaves a sum that started from +0.0 unchanged bit for
// bit (such a sum is never -0.0), so the result equals the sequential sum over the subset.
constexpr int kW = 64;
#define SA_WAVE_ROW_BEGIN(n)                        \
  const int32_t i = (int32_t)blockIdx.x;            \
  if (i >= (n)) return;                             \
  const int lane = threadIdx.x;

template <class F>
__device__ inline double wave_seq_sum(int32_t b, int32_t e, F term, double *lds) {
  const int lane = threadIdx.x;
  double acc = 0.0;
  for (int32_t c = b; c < e; c += kW) {
    const int32_t k = c + lane;
    lds[lane] = (k < e) ? term(k) : 0.0;
    __syncthreads();
    if (lane == 0) {
      const int32_t lim = min(kW, e - c);
      for (int32_t q = 0; q < lim; ++q) acc += lds[q];
    }
    __syncthreads();
  }
  if (lane == 0) lds[0] = acc;
  __syncthreads();
  const double r = lds[0];
  __syncthreads();
  return r;
}
__device__ inline int32_t wave_sum_i32(int32_t v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline bool wave_any(bool p) { return __ballot(p) != 0; }

// ---- validation -----------------------------------------------------------------------
// Entry-parallel (a block owns kBlock rows, whose row pointers it stages in LDS and checks
// first; coalesced reads of col and val): bit 1 a row pointer or column out of range or
// columns not ascending, 2 a row without its diagonal entry, 4 a non-finite value, 2048 row
// pointers that do not start at 0 and end at nnz.
__global__ __launch_bounds__(kBlock) void k_validate(int32_t n, int64_t nnz,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     int32_t *err) {
  __shared__ int32_t s_rp[kBlock + 1];
  __shared__ uint8_t s_diag[kBlock];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kBlock;
  const int32_t nr = (int32_t)min<int64_t>(kBlock, (int64_t)n - r0);
  if (blockIdx.x == 0 && t == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) atomicOr(err, 2048);
  if (t < nr) s_rp[t] = rp[r0 + t];
  if (t == 0) s_rp[nr] = rp[r0 + nr];
  s_diag[t] = 0;
  __syncthreads();
  // the block's row pointers: within [0, nnz] and not decreasing, else nothing is read
  const bool bad = t < nr && (s_rp[t] < 0 || s_rp[t + 1] < s_rp[t] || (int64_t)s_rp[t + 1] > nnz);
  if (__syncthreads_or(bad)) {
    if (t == 0) atomicOr(err, 1);
    return;
  }
  const int32_t e0 = s_rp[0], e1 = s_rp[nr];
  int32_t flags = 0;
  for (int32_t e = e0 + t; e < e1; e += kBlock) {
    int32_t lo = 0, hi = nr - 1;  // the entry's row: the last r with s_rp[r] <= e
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (s_rp[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int32_t c = col[e];
    if (c < 0 || c >= n) flags |= 1;
    if (e > s_rp[lo] && c <= col[e - 1]) flags |= 1;
    if (c == (int32_t)r0 + lo) s_diag[lo] = 1;
    if (val && !isfinite(val[e])) flags |= 4;
  }
  __syncthreads();
  if (t < nr && !s_diag[t]) flags |= 2;
  if (flags) atomicOr(err, flags);
}

// nnz: the length of col and val (rp[n] is checked against it on the device).
void validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                  const double *val, int32_t *err, hipStream_t s) {
  k_validate<<<grid_for(n), kBlock, 0, s>>>(n, nnz, rp, col, val, err);
  SA_LAUNCH_CHECK();
}
__global__ void k_find_diag(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                            double *dval) {
  SA_ROW_KERNEL_BEGIN(n)
  int32_t lo = rp[i], hi = rp[i + 1] - 1;
  double d = 0.0;
  while (lo <= hi) {
    int32_t mid = (lo + hi) >> 1;
    int32_t c = col[mid];
    if (c == i) {
      d = val[mid];
      break;
    }
    if (c < i) lo = mid + 1;
    else hi = mid - 1;
  }
  dval[i] = d;
}
void find_diag(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
               double *dval, hipStream_t s) {
  if (n <= 0) return;
  k_find_diag<<<grid_for(n), kBlock, 0, s>>>(n, rp, col, val, dval);
  SA_LAUNCH_CHECK();
}

// ---- strength (Sec. 1.1 criterion, evaluated squared) ----------------------------------
// Entry-parallel: block b owns rows [256 b, 256 b + 256), whose entries are one contiguous run;
// consecutive threads take consecutive entries (coalesced loads and mask stores), each finding
// its row by binary search over the block's row pointers in LDS; strong entries are counted per
// row with LDS integer atomics.
__global__ __launch_bounds__(kBlock) void k_strength(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ dval, double th2,
                                                     uint8_t *__restrict__ mask,
                                                     int32_t *__restrict__ scount) {
  __shared__ int32_t s_rp[kBlock + 1];
  __shared__ double s_d[kBlock];
  __shared__ int32_t s_cnt[kBlock];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kBlock;
  const int32_t nr = (int32_t)min<int64_t>(kBlock, (int64_t)n - r0);
  if (t < nr) {
    s_rp[t] = rp[r0 + t];
    s_d[t] = dval[r0 + t];
  }
  if (t == 0) s_rp[nr] = rp[r0 + nr];  // nr can be kBlock: no thread t == nr
  s_cnt[t] = 0;
  __syncthreads();
  const int32_t e0 = s_rp[0], e1 = s_rp[nr];
  for (int32_t e = e0 + t; e < e1; e += kBlock) {
    int32_t lo = 0, hi = nr - 1;  // the entry's row: the last r with s_rp[r] <= e
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (s_rp[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int32_t j = col[e];
    uint8_t m = 3;
    if (j != (int32_t)r0 + lo) {
      const double a = val[e];
      const double p = s_d[lo] * dval[j];
      const bool strong = (p > 0.0) && (a * a >= th2 * p);
      m = strong ? 1 : 0;
      if (strong) atomicAdd(&s_cnt[lo], 1);
    }
    mask[e] = m;
  }
  __syncthreads();
  if (t < nr) scount[r0 + t] = s_cnt[t];
}
__global__ __launch_bounds__(kW) void k_strength_w(int32_t n, const int32_t *rp,
                                                   const int32_t *col, const double *val,
                                                   const double *dval, double th2,
                                                   uint8_t *mask, int32_t *scount) {
  SA_WAVE_ROW_BEGIN(n)
  const double di = dval[i];
  int32_t cnt = 0;
  for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += kW) {
    const int32_t j = col[k];
    if (j == i) {
      mask[k] = 3;
      continue;
    }
    const double a = val[k];
    const double p = di * dval[j];
    const bool strong = (p > 0.0) && (a * a >= th2 * p);
    mask[k] = strong ? 1 : 0;
    cnt += strong;
  }
  cnt = wave_sum_i32(cnt);
  if (lane == 0) scount[i] = cnt;
}
void strength(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *dval, double th2, uint8_t *mask, int32_t *scount, bool wave,
              hipStream_t s) {
  if (n <= 0) return;
  if (wave) k_strength_w<<<(unsigned)n, kW, 0, s>>>(n, rp, col, val, dval, th2, mask, scount);
  else k_strength<<<grid_for(n), kBlock, 0, s>>>(n, rp, col, val, dval, th2, mask, scount);
  SA_LAUNCH_CHECK();
}

// ---- distance-Laplacian weights (Sec. 3.1) -------------------------------------------------
// The strength test can be taken on a Laplacian built from node coordinates instead of on A:
// same pattern, off-diagonal weight w = 1/d^P with d the distance (the squared distance d2
// summed over the coordinates in order from 0; P = 1: 1/sqrt(d2), both correctly rounded;
// P = 2: 1/d2), diagonal Ld[i] = the row's weights summed in ascending column order from 0.
// k_strength then runs on (w, Ld) unchanged: |L_ij| >= theta sqrt(L_ii L_jj) squared is
// w^2 >= theta^2 Ld_i Ld_j.  A zero (or NaN) distance between two connected nodes
// sets err bit `ebit`.
template <int D>
__device__ inline double dist2(const double *__restrict__ xyz, int32_t i, int32_t j) {
  double d2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double t = xyz[(int64_t)i * D + k] - xyz[(int64_t)j * D + k];
    d2 = d2 + t * t;
  }
  return d2;
}
template <int D, int P>
__global__ void k_distance_weights(int32_t n, const int32_t *rp, const int32_t *col,
                                   const double *__restrict__ xyz, double *w, double *Ld,
                                   int32_t *err, int32_t ebit) {
  SA_ROW_KERNEL_BEGIN(n)
  double s = 0.0;
  bool bad = false;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const int32_t j = col[k];
    if (j == i) {
      w[k] = 0.0;
      continue;
    }
    const double d2 = dist2<D>(xyz, i, j);
    bad |= !(d2 > 0.0);
    const double wk = P == 1 ? 1.0 / sqrt(d2) : 1.0 / d2;
    w[k] = wk;
    s = s + wk;
  }
  Ld[i] = s;
  if (bad) atomicOr(err, ebit);
}
template <int D>
static void distance_weights_dim(int32_t n, const int32_t *rp, const int32_t *col,
                                 const double *xyz, int32_t power, double *w, double *Ld,
                                 int32_t *err, int32_t ebit, hipStream_t s) {
  if (power == 1)
    k_distance_weights<D, 1><<<grid_for(n), kBlock, 0, s>>>(n, rp, col, xyz, w, Ld, err, ebit);
  else
    k_distance_weights<D, 2><<<grid_for(n), kBlock, 0, s>>>(n, rp, col, xyz, w, Ld, err, ebit);
}
void distance_weights(int32_t n, const int32_t *rp, const int32_t *col, const double *xyz,
                      int32_t dim, int32_t power, double *w, double *Ld, int32_t *err,
                      int32_t ebit, hipStream_t s) {
  if (n <= 0) return;
  if (power != 1 && power != 2) throw Error(SA_ERR_INVALID_ARG, "dist_power");
  switch (dim) {
    case 1: distance_weights_dim<1>(n, rp, col, xyz, power, w, Ld, err, ebit, s); break;
    case 2: distance_weights_dim<2>(n, rp, col, xyz, power, w, Ld, err, ebit, s); break;
    case 3: distance_weights_dim<3>(n, rp, col, xyz, power, w, Ld, err, ebit, s); break;
    default: throw Error(SA_ERR_INVALID_ARG, "coordinate dimension");
  }
  SA_LAUNCH_CHECK();
}

__global__ void k_check_finite(int64_t m, const double *x, int32_t *err, int32_t ebit) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m && !isfinite(x[i])) atomicOr(err, ebit);
}
void check_finite(const double *x, int64_t m, int32_t *err, int32_t ebit, hipStream_t s) {
  if (m <= 0) return;
  k_check_finite<<<grid_for(m), kBlock, 0, s>>>(m, x, err, ebit);
  SA_LAUNCH_CHECK();
}

// ---- coarse coordinates: aggregate centroids ---------------------------------------------
// Member lists by counting sort (count, scan, scatter, then each list sorted ascending), then
// one thread per aggregate sums its members' coordinates in ascending vertex order from 0
// and divides by the member count.
__global__ void k_count_members(int32_t n, const int32_t *agg, int32_t *cnt) {
  SA_ROW_KERNEL_BEGIN(n)
  if (agg[i] >= 0) atomicAdd(&cnt[agg[i]], 1);
}
__global__ void k_scatter_members(int32_t n, const int32_t *agg, int32_t *pos, int32_t *mem) {
  SA_ROW_KERNEL_BEGIN(n)
  if (agg[i] >= 0) mem[atomicAdd(&pos[agg[i]], 1)] = i;
}
// Member lists of the nc aggregates: mrp[nc+1] offsets into mem[n] (unaggregated vertices
// left out); members in scatter order, or ascending when `sorted`.
void member_lists(int32_t n, const int32_t *agg, int32_t nc, bool sorted, Arena &ar,
                  int32_t **mrp_out, int32_t **mem_out, hipStream_t s) {
  int32_t *cnt = ar.alloc<int32_t>(nc + 1);
  int32_t *mrp = ar.alloc<int32_t>(nc + 1);
  int32_t *mem = ar.alloc<int32_t>(n > 0 ? n : 1);
  fill_i32(cnt, 0, nc + 1, s);
  if (n > 0) {
    k_count_members<<<grid_for(n), kBlock, 0, s>>>(n, agg, cnt);
    SA_LAUNCH_CHECK();
  }
  exclusive_scan_i32(cnt, mrp, nc, s);
  SA_HIP(hipMemcpyAsync(cnt, mrp, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToDevice, s));
  if (n > 0) {
    k_scatter_members<<<grid_for(n), kBlock, 0, s>>>(n, agg, cnt, mem);
    SA_LAUNCH_CHECK();
  }
  if (sorted) sort_rows(nc, mrp, mem, nullptr, s);
  *mrp_out = mrp;
  *mem_out = mem;
}
__global__ void k_centroids(int32_t nc, int32_t dim, const int32_t *mrp, const int32_t *mem,
                            const double *__restrict__ xyz, double *cxyz) {
  SA_ROW_KERNEL_BEGIN(nc)
  const int32_t b = mrp[i], e = mrp[i + 1];
  for (int k = 0; k < dim; ++k) {
    double s = 0.0;
    for (int32_t q = b; q < e; ++q) s = s + xyz[(int64_t)mem[q] * dim + k];
    cxyz[(int64_t)i * dim + k] = s / (double)(e - b);
  }
}
void aggregate_centroids(int32_t n, const int32_t *agg, int32_t nc, const double *xyz,
                         int32_t dim, double *cxyz, hipStream_t s) {
  if (nc <= 0) return;
  Arena tmp;
  tmp.stream = s;
  int32_t *mrp, *mem;
  member_lists(n, agg, nc, true, tmp, &mrp, &mem, s);
  k_centroids<<<grid_for(nc), kBlock, 0, s>>>(nc, dim, mrp, mem, xyz, cxyz);
  SA_LAUNCH_CHECK();
}

// ---- aggregation graph G = S u S^T ------------------------------------------------------
__global__ void k_fill_strong(int32_t n, const int32_t *rp, const int32_t *col,
                              const uint8_t *mask, const int32_t *srp, int32_t *scol,
                              int32_t *tcnt) {
  SA_ROW_KERNEL_BEGIN(n)
  int32_t w = srp[i];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const uint8_t m = mask[k];
    if (m == 1 || m == 2) {
      scol[w++] = col[k];
      atomicAdd(&tcnt[col[k]], 1);
    }
  }
}
__global__ __launch_bounds__(kW) void k_fill_strong_w(int32_t n, const int32_t *rp,
                                                      const int32_t *col, const uint8_t *mask,
                                                      const int32_t *srp, int32_t *scol,
                                                      int32_t *tcnt) {
  SA_WAVE_ROW_BEGIN(n)
  int32_t w = srp[i];
  for (int32_t c = rp[i]; c < rp[i + 1]; c += kW) {
    const int32_t k = c + lane;
    bool st = false;
    int32_t j = 0;
    if (k < rp[i + 1]) {
      const uint8_t m = mask[k];
      st = (m == 1 || m == 2);
      j = col[k];
    }
    const unsigned long long bm = __ballot(st);
    if (st) {
      scol[w + __popcll(bm & ((1ull << lane) - 1ull))] = j;
      atomicAdd(&tcnt[j], 1);
    }
    w += __popcll(bm);
  }
}
__global__ void k_scatter_t(int32_t n, const int32_t *srp, const int32_t *scol, int32_t *tpos,
                            int32_t *tcol) {
  SA_ROW_KERNEL_BEGIN(n)
  for (int32_t k = srp[i]; k < srp[i + 1]; ++k) {
    int32_t p = atomicAdd(&tpos[scol[k]], 1);
    tcol[p] = i;
  }
}
__global__ void k_union(int32_t n, const int32_t *arp, const int32_t *acol, const int32_t *brp,
                        const int32_t *bcol, const int32_t *orp, int32_t *ocol, int32_t *ocnt) {
  SA_ROW_KERNEL_BEGIN(n)
  int32_t a = arp[i], ae = arp[i + 1], b = brp[i], be = brp[i + 1];
  int32_t w = orp ? orp[i] : 0;
  int32_t cnt = 0;
  while (a < ae || b < be) {
    int32_t v;
    if (b >= be || (a < ae && acol[a] < bcol[b])) v = acol[a++];
    else if (a >= ae || bcol[b] < acol[a]) v = bcol[b++];
    else {
      v = acol[a++];
      ++b;
    }
    if (ocol) ocol[w + cnt] = v;
    ++cnt;
  }
  if (ocnt) ocnt[i] = cnt;
}

int64_t strength_graph(int32_t n, const int32_t *rp, const int32_t *col, const uint8_t *mask,
                       const int32_t *scount, bool wave, Arena &ar, int32_t **grp_out,
                       int32_t **gcol_out, hipStream_t s) {
  Arena tmp;
  tmp.stream = s;
  int32_t *srp = tmp.alloc<int32_t>(n + 1);
  exclusive_scan_i32(scount, srp, n, s);
  const int32_t nnzS = read1(srp + n, s);
  int32_t *scol = tmp.alloc<int32_t>(nnzS);
  int32_t *tcnt = tmp.alloc<int32_t>(n + 1);
  fill_i32(tcnt, 0, n + 1, s);
  if (wave) k_fill_strong_w<<<(unsigned)n, kW, 0, s>>>(n, rp, col, mask, srp, scol, tcnt);
  else k_fill_strong<<<grid_for(n), kBlock, 0, s>>>(n, rp, col, mask, srp, scol, tcnt);
  SA_LAUNCH_CHECK();
  int32_t *trp = tmp.alloc<int32_t>(n + 1);
  exclusive_scan_i32(tcnt, trp, n, s);
  int32_t *tpos = tmp.alloc<int32_t>(n + 1);
  SA_HIP(hipMemcpyAsync(tpos, trp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  int32_t *tcol = tmp.alloc<int32_t>(nnzS);
  k_scatter_t<<<grid_for(n), kBlock, 0, s>>>(n, srp, scol, tpos, tcol);
  SA_LAUNCH_CHECK();
  sort_rows(n, trp, tcol, nullptr, s);
  int32_t *gcnt = tmp.alloc<int32_t>(n + 1);
  k_union<<<grid_for(n), kBlock, 0, s>>>(n, srp, scol, trp, tcol, nullptr, nullptr, gcnt);
  SA_LAUNCH_CHECK();
  int32_t *grp = ar.alloc<int32_t>(n + 1);
  exclusive_scan_i32(gcnt, grp, n, s);
  const int32_t nnzG = read1(grp + n, s);
  int32_t *gcol = ar.alloc<int32_t>(nnzG);
  k_union<<<grid_for(n), kBlock, 0, s>>>(n, srp, scol, trp, tcol, grp, gcol, nullptr);
  SA_LAUNCH_CHECK();
  *grp_out = grp;
  *gcol_out = gcol;
  return nnzG;
}

// ---- root selection: lexicographically-first distance-2 maximal independent set -----------
// key = (state, priority) with state IN < UNDECIDED < OUT in the top two bits, so the
// minimum key of a neighbourhood is its best vertex.  Per round: k1(v) = min key over N[v];
// then an undecided v with m = min k1 over N[v] (the minimum over the distance-2 ball)
// leaves as OUT when m is an IN key (a root within distance 2) and enters as IN when m is its
// own key (it has the best priority among undecided vertices within distance 2).  This
// reproduces the sequential greedy root choice in priority order exactly.
//
// Rounds are event driven: k1(u) is recomputed only in a round after some key in N[u]
// changed, and an undecided v re-takes its decision only in a round in which some k1 in N[v]
// changed; any other vertex would compute the value (or the "wait") it already holds, so the
// selection is the same as re-evaluating every vertex every round.  The triggers are 1-byte
// round stamps (round number mod 256): pass 2 stamps N[v] u {v} for pass 1 of the next round
// when v's key changes, pass 1 stamps N[u] u {u} for pass 2 of the same round when k1(u)
// changes.  A stale stamp that matches after wrap-around only costs a needless re-evaluation.
// Round 0 evaluates everything (all stamps start at 0).  A round that changes no key ends
// the selection: nothing can change after it.  Natural order uses 32-bit keys
// (state << 30 | index); hashed order 64-bit keys (state << 62 | hash30 << 32 | index).
// Levels with high average degree use one wavefront per vertex.
template <class K>
struct KeyT;
template <>
struct KeyT<uint32_t> {
  static constexpr uint32_t In = 0, Und = 1u << 30, Out = 2u << 30, Mask = 3u << 30;
};
template <>
struct KeyT<uint64_t> {
  static constexpr uint64_t In = 0, Und = 1ull << 62, Out = 2ull << 62, Mask = 3ull << 62;
};

__device__ inline uint64_t splitmix64_dev(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline uint64_t stream_key_dev(int stream, int level, int64_t i) {
  return ((uint64_t)stream << 56) | ((uint64_t)level << 40) | (uint64_t)i;
}

// A vertex without neighbours is decided at once: nothing near it can ever be aggregated, so
// the sequential rule makes it a root whatever its priority (singletons), or it is left out.
// Its key never enters another vertex's neighbourhood minimum.
template <class K>
__global__ void k_mis_init(int32_t n, const int32_t *grp, int32_t order, uint64_t seed,
                           int32_t level, bool singletons, K *key, uint8_t *st1, uint8_t *st2) {
  SA_ROW_KERNEL_BEGIN(n)
  K pri = (K)i;
  if (order == 1)
    pri = (K)((((uint64_t)splitmix64_dev(seed, stream_key_dev(2, level, i)) >> 34) << 32) |
              (uint64_t)i);
  const bool open = grp[i + 1] > grp[i];
  key[i] = (open ? KeyT<K>::Und : singletons ? KeyT<K>::In : KeyT<K>::Out) | pri;
  st1[i] = 0;
  st2[i] = 0;
}

// Stamps i and every vertex of gcol[b..e) with s: 8 independent index loads, then 8 stores
// (the last index repeated past the end: the same byte stored again).
__device__ inline void stamp_ball(const int32_t *__restrict__ gcol, int32_t b, int32_t e,
                                  int32_t i, uint8_t *__restrict__ st, uint8_t s) {
  st[i] = s;
  for (int32_t k = b; k < e; k += 8) {
    int32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = gcol[min(k + q, e - 1)];
#pragma unroll
    for (int q = 0; q < 8; ++q) st[c[q]] = s;
  }
}

// Pass 1 for one stamped vertex i (thread per vertex): k1(i) = min key over N[i] u {i}; a
// changed minimum stamps N[i] u {i} for pass 2.
template <class K>
__device__ __forceinline__ void mis1_vertex(int32_t i, const int32_t *__restrict__ grp,
                                            const int32_t *__restrict__ gcol,
                                            const K *__restrict__ key, K *__restrict__ k1,
                                            uint8_t *__restrict__ st2, uint8_t sr, bool first) {
  const int32_t b = grp[i], e = grp[i + 1];
  K m = key[i];
  const K old = first ? m : k1[i];
  // neighbours 8 at a time: all indices, then all keys, as independent loads (i itself
  // past the end of the list, harmless in the minimum); the first 8 indices are kept for
  // the stamps
  int32_t c0[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) c0[q] = i;
  for (int32_t k = b; k < e; k += 8) {
    int32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t g = gcol[min(k + q, e - 1)];  // in bounds even if loaded eagerly
      c[q] = (k + q < e) ? g : i;
    }
    K kv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) kv[q] = key[c[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q) m = kv[q] < m ? kv[q] : m;
    if (k == b) {
#pragma unroll
      for (int q = 0; q < 8; ++q) c0[q] = c[q];
    }
  }
  if (!first && m != old) {
    if (e - b <= 8) {
      st2[i] = sr;
#pragma unroll
      for (int q = 0; q < 8; ++q) st2[c0[q]] = sr;
    } else {
      stamp_ball(gcol, b, e, i, st2, sr);
    }
  }
  k1[i] = m;
}

constexpr int kMisV = 4;                // vertices per thread on large levels
constexpr int64_t kMisVMinN = 524288;   // from this level size on

// Pass 1 of round r (stamp sr): k1(u) = min key over N[u] for stamped u.  V > 1 (thread
// per vertex only): each thread takes V vertices, for levels with many vertices.
template <class K, bool WAVE, int V = 1>
__global__ void k_mis_pass1(int32_t n, const int32_t *__restrict__ grp,
                            const int32_t *__restrict__ gcol, const K *__restrict__ key,
                            K *__restrict__ k1, const uint8_t *__restrict__ st1,
                            uint8_t *__restrict__ st2, uint8_t sr, bool first,
                            const int32_t *__restrict__ prev, int32_t *__restrict__ cur,
                            uint32_t *hstat, uint32_t tag) {
  static_assert(!(WAVE && V > 1), "a wavefront per vertex takes one vertex");
  // one thread clears this round's flag (pass 2 raises it) and posts the previous round's
  // outcome to the host's status word: tag | 1 if it changed a key, tag | 2 if not
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *cur = 0;
    if (hstat)
      __hip_atomic_store(hstat, tag | (*prev == 0 ? 2u : 1u), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  }
  // the stamp and the previous round's flag are read together (one round trip); a round
  // whose predecessor changed nothing exits
  if (WAVE) {
    const int lane = threadIdx.x & 63;
    const int64_t v64 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (v64 >= n) return;
    const int32_t v = (int32_t)v64;
    const uint8_t st = st1[v];
    if ((prev && *prev == 0) | (st != sr)) return;  // wave-uniform
    const int32_t b = grp[v], e = grp[v + 1];
    K m = (lane == 0) ? key[v] : ~(K)0;
    for (int32_t k = b + lane; k < e; k += 64) {
      const K ku = key[gcol[k]];
      m = ku < m ? ku : m;
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const K o = __shfl_xor(m, off, 64);
      m = o < m ? o : m;
    }
    const K old = first ? m : k1[v];  // read by every lane before lane 0 stores
    if (lane == 0) k1[v] = m;
    if (!first && m != old) {
      for (int32_t k = b + lane; k < e; k += 64) st2[gcol[k]] = sr;
      if (lane == 0) st2[v] = sr;
    }
  } else if (V == 1) {
    SA_ROW_KERNEL_BEGIN(n)
    const uint8_t st = st1[i];
    if ((prev && *prev == 0) | (st != sr)) return;
    mis1_vertex<K>(i, grp, gcol, key, k1, st2, sr, first);
  } else {
    // V vertices per thread at a stride of the grid's thread count (neighbouring vertices,
    // which tend to be stamped together, stay on different lanes); their stamps and the
    // previous round's flag are read together
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint8_t st[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t v = t + j * nt;
      st[j] = v < n ? st1[v] : (uint8_t)(sr + 1);
    }
    if (prev && *prev == 0) return;
#pragma unroll 1
    for (int j = 0; j < V; ++j)
      if (st[j] == sr) mis1_vertex<K>((int32_t)(t + j * nt), grp, gcol, key, k1, st2, sr, first);
  }
}

// Pass 2 for one stamped vertex i (thread per vertex): an undecided i takes m = min k1 over
// N[i] u {i}; an IN key there makes it OUT, its own key makes it IN.  A change stamps
// N[i] u {i} with srn and raises the round's flag.
template <class K>
__device__ __forceinline__ void mis2_vertex(int32_t i, const int32_t *__restrict__ grp,
                                            const int32_t *__restrict__ gcol,
                                            const K *__restrict__ k1, K *__restrict__ key,
                                            uint8_t *__restrict__ st1, uint8_t srn,
                                            int32_t *__restrict__ flag) {
  // the key, the row range and k1 together (the test below uses them all, so none of the
  // loads waits for the state test)
  const K me = key[i];
  K m = k1[i];
  const int32_t b = grp[i], e = grp[i + 1];
  if (((me & KeyT<K>::Mask) != KeyT<K>::Und) | (e < b)) return;
  int32_t c0[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) c0[q] = i;
  for (int32_t k = b; k < e; k += 8) {
    int32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t g = gcol[min(k + q, e - 1)];  // in bounds even if loaded eagerly
      c[q] = (k + q < e) ? g : i;
    }
    K kv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) kv[q] = k1[c[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q) m = kv[q] < m ? kv[q] : m;
    if (k == b) {
#pragma unroll
      for (int q = 0; q < 8; ++q) c0[q] = c[q];
    }
  }
  const K pri = me & ~KeyT<K>::Mask;
  K nk = me;
  if ((m & KeyT<K>::Mask) == KeyT<K>::In) nk = KeyT<K>::Out | pri;
  else if (m == me) nk = KeyT<K>::In | pri;
  if (nk != me) {
    key[i] = nk;
    if (e - b <= 8) {
      st1[i] = srn;
#pragma unroll
      for (int q = 0; q < 8; ++q) st1[c0[q]] = srn;
    } else {
      stamp_ball(gcol, b, e, i, st1, srn);
    }
    *flag = 1;
  }
}

// Pass 2 of round r: stamped undecided v takes m = min k1 over N[v]; an IN key there makes v
// OUT, its own key makes it IN.  A change stamps N[v] u {v} with the next round's stamp srn
// and raises the round's flag.  V > 1: V vertices per thread, as in pass 1.
template <class K, bool WAVE, int V = 1>
__global__ void k_mis_pass2(int32_t n, const int32_t *__restrict__ grp,
                            const int32_t *__restrict__ gcol, const K *__restrict__ k1,
                            K *__restrict__ key, const uint8_t *__restrict__ st2,
                            uint8_t *__restrict__ st1, uint8_t sr, uint8_t srn,
                            int32_t *__restrict__ flag, const int32_t *__restrict__ prev) {
  static_assert(!(WAVE && V > 1), "a wavefront per vertex takes one vertex");
  if (WAVE) {
    const int lane = threadIdx.x & 63;
    const int64_t v64 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (v64 >= n) return;
    const int32_t v = (int32_t)v64;
    const uint8_t st = st2[v];
    if ((prev && *prev == 0) | (st != sr)) return;  // wave-uniform
    const K me = key[v];
    const int32_t b = grp[v], e = grp[v + 1];
    if (((me & KeyT<K>::Mask) != KeyT<K>::Und) | (e < b)) return;  // wave-uniform
    K m = (lane == 0) ? k1[v] : ~(K)0;
    for (int32_t k = b + lane; k < e; k += 64) {
      const K ku = k1[gcol[k]];
      m = ku < m ? ku : m;
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const K o = __shfl_xor(m, off, 64);
      m = o < m ? o : m;
    }
    const K pri = me & ~KeyT<K>::Mask;
    K nk = me;
    if ((m & KeyT<K>::Mask) == KeyT<K>::In) nk = KeyT<K>::Out | pri;
    else if (m == me) nk = KeyT<K>::In | pri;
    if (nk != me) {  // wave-uniform
      for (int32_t k = b + lane; k < e; k += 64) st1[gcol[k]] = srn;
      if (lane == 0) {
        key[v] = nk;
        st1[v] = srn;
        *flag = 1;
      }
    }
  } else if (V == 1) {
    SA_ROW_KERNEL_BEGIN(n)
    const uint8_t st = st2[i];
    if ((prev && *prev == 0) | (st != sr)) return;
    mis2_vertex<K>(i, grp, gcol, k1, key, st1, srn, flag);
  } else {
    // V vertices per thread at a stride of the grid's thread count, as in pass 1
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint8_t st[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t v = t + j * nt;
      st[j] = v < n ? st2[v] : (uint8_t)(sr + 1);
    }
    if (prev && *prev == 0) return;
#pragma unroll 1
    for (int j = 0; j < V; ++j)
      if (st[j] == sr) mis2_vertex<K>((int32_t)(t + j * nt), grp, gcol, k1, key, st1, srn, flag);
  }
}

// ---- root selection in one workgroup --------------------------------------------------------
// On levels of at most kMisWgMaxN vertices, every round after the first runs inside a single
// workgroup of kMisWg threads: the same two passes, triggers and early end as above, with
// __syncthreads() between passes instead of kernel boundaries.  The triggered vertices of a
// pass are kept as lists; a vertex enters a list once, through a bit in an LDS bitmap (bm1
// for pass-1 lists, bm2 for pass-2 lists) that is set with an atomic or and cleared when the
// entry is taken, so list lengths stay within n.  Round 1's pass-1 list is read from the byte
// stamps that the grid round 0 left (value 1).  G lanes share a vertex (lane j takes entries
// j, j+G, ...).  The round count and the keys equal the grid path's.
// result[0] = the first round that changed nothing, result[1] = 1 if max_rounds was reached;
// the same word goes to the host-mapped post (bit 31 set on that error).
constexpr int kMisWg = 1024;
constexpr int64_t kMisWgMaxN = 4096;  // default level size limit (SAAMG_MIS_WG_MAX_N)
constexpr int64_t kMisWgLdsMaxN = 131072;  // the bitmaps' limit: 2 x 16 KiB of LDS
constexpr size_t kMisWgKeyLds = 64 << 10;  // keys and k1 in LDS up to this many bytes

// Appends the slots q with take[q] of every active lane to list: one LDS atomic per
// wavefront, slots in lane-major order of the ballots.
template <int Q>
__device__ inline void wave_append(const int32_t (&w)[Q], const bool (&take)[Q],
                                   int32_t *list, int32_t *cnt) {
  uint32_t off[Q];
  uint32_t total = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint64_t m = __ballot(take[q]);
    off[q] = total + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    total += (uint32_t)__popcll(m);
  }
  if (total == 0) return;  // uniform over the active lanes
  const uint64_t act = __ballot(true);
  int32_t base = 0;
  if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1)
    base = atomicAdd(cnt, (int32_t)total);
  base = __builtin_amdgcn_readfirstlane(base);
#pragma unroll
  for (int q = 0; q < Q; ++q)
    if (take[q]) list[base + (int32_t)off[q]] = w[q];
}

// KL: the keys and k1 live in LDS during the rounds (after the bitmaps, at an 8-byte
// boundary), read from and written back to global memory around them.
template <class K, int G, bool KL>
__global__ __launch_bounds__(kMisWg) void k_mis_rounds_wg(
    int32_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ gcol, K *gkey,
    K *gk1, const uint8_t *__restrict__ st1, const int32_t *__restrict__ flag0, int32_t *l1,
    int32_t *l2, int32_t max_rounds, int32_t *result, uint32_t *hpost) {
  extern __shared__ uint64_t lds_wg[];  // 8-byte aligned: the keys may be 64-bit
  uint32_t *bm = reinterpret_cast<uint32_t *>(lds_wg);  // bm1 = bm[0, nwb), bm2 = bm[nwb, 2 nwb)
  __shared__ int32_t c1, c2, chg[2];
  const int tid = threadIdx.x;
  const int j = tid % G;     // lane within the vertex's group
  const int grp0 = tid / G;  // group number
  constexpr int kGroups = kMisWg / G;
  const int32_t nwb = (n + 31) >> 5;
  uint32_t *bm1 = bm, *bm2 = bm + nwb;
  K *key = gkey, *k1 = gk1;
  if constexpr (KL) {
    key = reinterpret_cast<K *>(bm + ((2 * nwb + 1) & ~1));
    k1 = key + n;
    for (int32_t v = tid; v < n; v += kMisWg) {
      key[v] = gkey[v];
      k1[v] = gk1[v];
    }
  }
  for (int32_t w = tid; w < 2 * nwb; w += kMisWg) bm[w] = 0u;
  if (tid == 0) {
    c1 = 0;
    c2 = 0;
    chg[0] = 0;
    chg[1] = 0;
  }
  __syncthreads();
  // min of x over v (lane 0) and N[v] = gcol[b..e), 8 independent loads per step
  auto ball_min = [&](const K *x, int32_t v, int32_t b, int32_t e) {
    K m = (j == 0) ? x[v] : ~(K)0;
    for (int32_t k = b + j; k < e; k += 8 * G) {
      int32_t c[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) c[q] = gcol[min(k + q * G, e - 1)];
      K kv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) kv[q] = x[c[q]];
#pragma unroll
      for (int q = 0; q < 8; ++q) m = kv[q] < m ? kv[q] : m;
    }
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
      const K o = __shfl_xor(m, off, G);
      m = o < m ? o : m;
    }
    return m;
  };
  // lists v and N[v] (slot b-1 stands for v) unless their bit is set; slots past the end
  // take a no-op or on v's word
  auto push_ball = [&](int32_t v, int32_t b, int32_t e, uint32_t *bmx, int32_t *list,
                       int32_t *cnt) {
    for (int32_t k = b - 1 + j; k < e; k += 8 * G) {
      int32_t w[8];
      bool take[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t kk = k + q * G;
        w[q] = (kk < b || kk >= e) ? v : gcol[kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t bit = (k + q * G < e) ? 1u << (w[q] & 31) : 0u;
        take[q] = bit != 0u && (atomicOr(bmx + (w[q] >> 5), bit) & bit) == 0u;
      }
      wave_append<8>(w, take, list, cnt);
    }
  };
  uint32_t used = 0, err = 0;
  if (*flag0 != 0) {
    // round 1's pass-1 list: the vertices stamped 1 by round 0 (4 stamps per word; the byte
    // array is padded to a multiple of 16)
    const int32_t nw = (n + 3) >> 2;
    for (int32_t w0 = tid; w0 - tid < nw; w0 += kMisWg) {  // every lane runs every step
      const uint32_t word = w0 < nw ? reinterpret_cast<const uint32_t *>(st1)[w0] : 0u;
      int32_t w[4];
      bool take[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        w[q] = 4 * w0 + q;
        take[q] = w[q] < n && ((word >> (8 * q)) & 0xffu) == 1u;
      }
      wave_append<4>(w, take, l1, &c1);
    }
    __syncthreads();
    for (uint32_t r = 1;; ++r) {
      // pass 1: k1(u) = min key over N[u] for listed u; a change lists N[u] u {u} for pass 2
      const int32_t n1 = c1;
      for (int32_t idx = grp0; idx < n1; idx += kGroups) {
        const int32_t u = l1[idx];
        if (j == 0) atomicAnd(bm1 + (u >> 5), ~(1u << (u & 31)));
        const int32_t b = grp[u], e = grp[u + 1];
        const K old = k1[u];
        const K m = ball_min(key, u, b, e);
        if (j == 0) k1[u] = m;
        if (m != old) push_ball(u, b, e, bm2, l2, &c2);
      }
      __syncthreads();
      const int32_t n2 = c2;
      __syncthreads();  // every thread holds n1 and n2: both counters may restart
      if (tid == 0) {
        c1 = 0;
        c2 = 0;
        chg[r & 1] = 0;
      }
      __syncthreads();
      // pass 2: a listed undecided v takes m = min k1 over N[v]; a change lists N[v] u {v}
      // for pass 1 of the next round
      for (int32_t idx = grp0; idx < n2; idx += kGroups) {
        const int32_t v = l2[idx];
        if (j == 0) atomicAnd(bm2 + (v >> 5), ~(1u << (v & 31)));
        const K me = key[v];
        const int32_t b = grp[v], e = grp[v + 1];
        if ((me & KeyT<K>::Mask) != KeyT<K>::Und) continue;  // group-uniform
        const K m = ball_min(k1, v, b, e);
        const K pri = me & ~KeyT<K>::Mask;
        K nk = me;
        if ((m & KeyT<K>::Mask) == KeyT<K>::In) nk = KeyT<K>::Out | pri;
        else if (m == me) nk = KeyT<K>::In | pri;
        if (nk != me) {  // group-uniform
          if (j == 0) {
            key[v] = nk;
            chg[r & 1] = 1;
          }
          push_ball(v, b, e, bm1, l1, &c1);
        }
      }
      __syncthreads();
      if (chg[r & 1] == 0) {  // workgroup-uniform
        used = r;
        break;
      }
      if ((int64_t)r >= (int64_t)max_rounds) {
        used = r;
        err = 1;
        break;
      }
    }
  }
  if constexpr (KL) {  // the keys back to global memory (k1 is not read after the rounds)
    __syncthreads();
    for (int32_t v = tid; v < n; v += kMisWg) gkey[v] = key[v];
  }
  if (tid == 0) {
    result[0] = (int32_t)used;
    result[1] = (int32_t)err;
    if (hpost)
      __hip_atomic_store(hpost, used | (err << 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Largest row length of a CSR (two-stage maximum, no contended atomics).
__global__ void k_rowlen_max_stage(int32_t n, const int32_t *rp, int32_t *part) {
  __shared__ int32_t sh[kBlock];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  sh[threadIdx.x] = (i < n) ? rp[i + 1] - rp[i] : 0;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_max_i32(int32_t n, const int32_t *a, int32_t *out) {
  __shared__ int32_t sh[kBlock];
  int32_t m = 0;
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) m = max(m, a[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}
int32_t max_row_length(int32_t n, const int32_t *rp, hipStream_t s) {
  if (n <= 0) return 0;
  const unsigned nb = grid_for(n);
  int32_t *part = (int32_t *)dev_alloc(sizeof(int32_t) * (nb + 1), s);
  k_rowlen_max_stage<<<nb, kBlock, 0, s>>>(n, rp, part);
  k_max_i32<<<1, kBlock, 0, s>>>((int32_t)nb, part, part + nb);
  SA_LAUNCH_CHECK();
  const int32_t m = read1(part + nb, s);
  dev_free(part, s);
  return m;
}

template <class K>
__global__ void k_roots(int32_t n, const K *key, int32_t *isr) {
  SA_ROW_KERNEL_BEGIN(n)
  isr[i] = ((key[i] & KeyT<K>::Mask) == KeyT<K>::In) ? 1 : 0;
}
template <class K>
__global__ void k_agg_phase1(int32_t n, const int32_t *grp, const int32_t *gcol, const K *key,
                             const int32_t *rid, int32_t *agg1, uint8_t *is_root,
                             int32_t *root_vertex) {
  SA_ROW_KERNEL_BEGIN(n)
  int32_t a = -1;
  const bool root = (key[i] & KeyT<K>::Mask) == KeyT<K>::In;
  if (root) {
    a = rid[i];
    root_vertex[a] = i;
  } else {
    for (int32_t k = grp[i]; k < grp[i + 1]; ++k) {
      const int32_t u = gcol[k];
      if ((key[u] & KeyT<K>::Mask) == KeyT<K>::In) {
        a = rid[u];
        break;
      }
    }
  }
  agg1[i] = a;
  is_root[i] = root ? 1 : 0;
}
// Leftover vertices join the phase-1 aggregate with the most strong connections to them,
// ties to the smaller aggregate number (a total order on the candidates: the choice does not
// depend on the order they are looked at in).
// Rows of up to R entries: the neighbours' phase-1 aggregates are loaded once, in one batch
// (-1 past the end of the row), and counted in registers.
template <int R>
__device__ __forceinline__ int32_t agg_join_regs(int32_t b, int32_t e,
                                                 const int32_t *__restrict__ gcol,
                                                 const int32_t *__restrict__ agg1) {
  int32_t g[R], c[R];
#pragma unroll
  for (int q = 0; q < R; ++q) g[q] = gcol[min(b + q, e - 1)];
#pragma unroll
  for (int q = 0; q < R; ++q) c[q] = (b + q < e) ? agg1[g[q]] : -1;
  int32_t best = -1, bestc = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (c[k] < 0) continue;
    int32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) cnt += (c[q] == c[k]);
    if (cnt > bestc || (cnt == bestc && c[k] < best)) {
      best = c[k];
      bestc = cnt;
    }
  }
  return best;
}

__global__ void k_agg_phase2(int32_t n, const int32_t *grp, const int32_t *gcol,
                             const int32_t *agg1, int32_t *agg) {
  SA_ROW_KERNEL_BEGIN(n)
  int32_t a = agg1[i];
  const int32_t b = grp[i], e = grp[i + 1];
  if (a < 0 && e > b) {
    if (e - b <= 8) {
      a = agg_join_regs<8>(b, e, gcol, agg1);
    } else if (e - b <= 32) {
      a = agg_join_regs<32>(b, e, gcol, agg1);
    } else {
      int32_t best = -1, bestc = 0;
      for (int32_t k = b; k < e; ++k) {
        const int32_t c = agg1[gcol[k]];
        if (c < 0) continue;
        int32_t cnt = 0;
        for (int32_t q = b; q < e; ++q) cnt += (agg1[gcol[q]] == c);
        if (cnt > bestc || (cnt == bestc && c < best)) {
          best = c;
          bestc = cnt;
        }
      }
      a = best;
    }
  }
  agg[i] = a;
}

template <class K>
static int32_t aggregate_impl(int32_t n, int64_t nnzG, const int32_t *grp, const int32_t *gcol,
                              int32_t order, uint64_t seed, int32_t level, bool singletons,
                              int32_t *agg,
                              uint8_t *is_root, Arena &ar, int32_t **root_vertex,
                              int32_t *rounds_out, hipStream_t s) {
  Arena tmp;
  tmp.stream = s;
  K *key = tmp.alloc<K>(n);
  K *k1 = tmp.alloc<K>(n);
  uint8_t *st1 = tmp.alloc<uint8_t>((n + 15) & ~15);  // padded for word reads
  uint8_t *st2 = tmp.alloc<uint8_t>((n + 15) & ~15);
  // levels up to wg_max_n vertices run the rounds after the first in one workgroup
  int64_t wg_max_n = kMisWgMaxN;
  if (const char *e = std::getenv("SAAMG_MIS_WG_MAX_N")) wg_max_n = std::atoll(e);
  const bool one_wg = nnzG > 0 && n <= std::min(wg_max_n, kMisWgLdsMaxN);
  k_mis_init<K><<<grid_for(n), kBlock, 0, s>>>(n, grp, order, seed, level, singletons, key, st1,
                                               st2);
  SA_LAUNCH_CHECK();
  // Rounds are launched back to back, at most kAhead past the last round whose outcome the
  // host has seen.  Pass 1 of round r+1 posts round r's outcome into a pinned status ring
  // (slot r mod kRing, tagged with r); the first round that changed nothing ends the
  // selection, and the rounds still queued behind it exit at once.  Device flags live in a
  // ring of the same size: pass 1 of round r clears slot r, pass 2 raises it.  If a status
  // word is not seen within spin_ns (20 ms; the environment variable SAAMG_STATUS_SPIN_NS
  // overrides it, 0 taking the fallback at every wait), the stream is synchronised and the
  // device flags read instead, so the outcome never depends on the host mapping alone.
  constexpr int kRing = 256, kAhead = 6;
  int64_t spin_ns = 20000000;
  if (const char *e = std::getenv("SAAMG_STATUS_SPIN_NS")) spin_ns = std::atoll(e);
  // every round before the last decides at least one vertex, so this bound is never reached
  const int64_t cap = (int64_t)n + 2 + 2 * kAhead;
  int32_t *flags = tmp.alloc<int32_t>(kRing);
  volatile uint32_t *hs = (volatile uint32_t *)pinned_status(sizeof(uint32_t) * kRing);
  for (int q = 0; q < kRing; ++q) hs[q] = ~0u;
  uint32_t *hs_dev = nullptr;
  SA_HIP(hipHostGetDevicePointer((void **)&hs_dev, (void *)hs, 0));
  const int32_t maxdeg = max_row_length(n, grp, s);
  const bool wave = maxdeg > 64 || nnzG > 24 * (int64_t)n;
  const unsigned g = wave ? grid_for((int64_t)n * 64) : grid_for(n);
  // large thread-per-vertex levels: kMisV vertices per thread (grid gv), fewer workgroups to
  // dispatch per pass; SAAMG_MIS_V_MIN_N overrides the level size from which they are used
  int64_t v_min_n = kMisVMinN;
  if (const char *e = std::getenv("SAAMG_MIS_V_MIN_N")) v_min_n = std::atoll(e);
  const unsigned gv =
      (!wave && n >= v_min_n) ? (unsigned)ceil_div(n, (int64_t)kBlock * kMisV) : 0u;
  auto launch_round = [&](int64_t r) {
    const uint8_t sr = (uint8_t)(r & 255), srn = (uint8_t)((r + 1) & 255);
    const bool first = r == 0;
    const int32_t *prev = first ? nullptr : flags + ((r - 1) & (kRing - 1));
    int32_t *cur = flags + (r & (kRing - 1));
    uint32_t *post = first ? nullptr : hs_dev + ((r - 1) & (kRing - 1));
    const uint32_t tag = (uint32_t)(r - 1) << 2;
    if (wave) {
      k_mis_pass1<K, true><<<g, kBlock, 0, s>>>(n, grp, gcol, key, k1, st1, st2, sr, first,
                                                 prev, cur, post, tag);
      k_mis_pass2<K, true><<<g, kBlock, 0, s>>>(n, grp, gcol, k1, key, st2, st1, sr, srn, cur,
                                                 prev);
    } else if (gv > 0) {
      k_mis_pass1<K, false, kMisV><<<gv, kBlock, 0, s>>>(n, grp, gcol, key, k1, st1, st2, sr,
                                                         first, prev, cur, post, tag);
      k_mis_pass2<K, false, kMisV><<<gv, kBlock, 0, s>>>(n, grp, gcol, k1, key, st2, st1, sr,
                                                         srn, cur, prev);
    } else {
      k_mis_pass1<K, false><<<g, kBlock, 0, s>>>(n, grp, gcol, key, k1, st1, st2, sr, first,
                                                  prev, cur, post, tag);
      k_mis_pass2<K, false><<<g, kBlock, 0, s>>>(n, grp, gcol, k1, key, st2, st1, sr, srn,
                                                  cur, prev);
    }
    SA_LAUNCH_CHECK();
  };
  int64_t launched = 0, seen = 0;  // rounds launched; rounds whose outcome is known
  int32_t used = 0;
  bool done = nnzG == 0;
  int32_t *wg_result = nullptr;
  if (one_wg) {
    // round 0 on the grid (every vertex), the rest in one workgroup
    wg_result = tmp.alloc<int32_t>(2);
    int32_t *l12 = tmp.alloc<int32_t>(2 * (int64_t)n);
    launch_round(0);
    const int32_t max_rounds = (int32_t)std::min<int64_t>((int64_t)n + 2, INT32_MAX);
    // rows past 16 entries: 4 lanes per vertex
    const size_t bits = sizeof(uint32_t) * (size_t)((2 * ((n + 31) / 32) + 1) & ~1);
    // the keys and k1 go to LDS too while they fit kMisWgKeyLds bytes
    const size_t keys = 2 * sizeof(K) * (size_t)n;
    const bool kl = keys <= kMisWgKeyLds;
    const size_t lds = bits + (kl ? keys : 0);
    auto go = [&](auto g, auto klc) {
      constexpr int G = decltype(g)::value;
      constexpr bool KL = decltype(klc)::value;
      k_mis_rounds_wg<K, G, KL><<<1, kMisWg, lds, s>>>(n, grp, gcol, key, k1, st1, flags, l12,
                                                       l12 + n, max_rounds, wg_result, hs_dev);
    };
    using G1 = std::integral_constant<int, 1>;
    using G4 = std::integral_constant<int, 4>;
    if (maxdeg > 16) {
      if (kl) go(G4{}, std::true_type{});
      else go(G4{}, std::false_type{});
    } else {
      if (kl) go(G1{}, std::true_type{});
      else go(G1{}, std::false_type{});
    }
    SA_LAUNCH_CHECK();
    done = true;
  }
  auto wait_from = std::chrono::steady_clock::now();
  while (!done) {
    // round `seen`'s status is posted by pass 1 of round seen+1
    if (launched >= seen + 2) {
      const uint32_t v = hs[seen & (kRing - 1)];
      if ((v & ~3u) == ((uint32_t)seen << 2) && (v & 3u) != 0 && v != ~0u) {
        if ((v & 3u) == 2u) {
          used = (int32_t)seen;
          done = true;
        } else {
          ++seen;
        }
        wait_from = std::chrono::steady_clock::now();
        continue;
      }
    }
    if (launched < seen + kAhead) {
      if (launched >= cap) throw Error(SA_ERR_COARSEN_STALLED, "root selection did not end");
      launch_round(launched++);
      continue;
    }
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration_cast<std::chrono::nanoseconds>(now - wait_from).count() <
        spin_ns)
      continue;
    // status not seen in time: every launched round's flag is final when the readback's copy
    // runs (after them on the stream)
    int32_t hf[kRing];
    readback(hf, flags, sizeof(hf), s);
    for (; seen < launched && !done; ++seen)
      if (hf[seen & (kRing - 1)] == 0) {
        used = (int32_t)seen;
        done = true;
      }
    if (done) break;
    wait_from = std::chrono::steady_clock::now();
  }
  int32_t *isr = tmp.alloc<int32_t>(n + 1);
  k_roots<K><<<grid_for(n), kBlock, 0, s>>>(n, key, isr);
  SA_LAUNCH_CHECK();
  int32_t *rid = tmp.alloc<int32_t>(n + 1);
  exclusive_scan_i32(isr, rid, n, s);
  const int32_t nc = read1(rid + n, s);  // returns once the stream's work so far is done
  if (one_wg) {
    // the workgroup's outcome, posted to the host-mapped word (read back if it is not seen)
    uint32_t v = hs[0];
    if (v == ~0u) {
      int32_t r2[2];
      readback(r2, wg_result, sizeof(r2), s);
      v = (uint32_t)r2[0] | ((uint32_t)r2[1] << 31);
    }
    if (v >> 31) throw Error(SA_ERR_COARSEN_STALLED, "root selection did not end");
    used = (int32_t)v;
  }
  if (rounds_out) *rounds_out = used;
  int32_t *rv = ar.alloc<int32_t>(nc > 0 ? nc : 1);
  int32_t *agg1 = tmp.alloc<int32_t>(n);
  k_agg_phase1<K><<<grid_for(n), kBlock, 0, s>>>(n, grp, gcol, key, rid, agg1, is_root, rv);
  SA_LAUNCH_CHECK();
  k_agg_phase2<<<grid_for(n), kBlock, 0, s>>>(n, grp, gcol, agg1, agg);
  SA_LAUNCH_CHECK();
  *root_vertex = rv;
  return nc;
}

int32_t aggregate(int32_t n, int64_t nnzG, const int32_t *grp, const int32_t *gcol,
                  int32_t order, uint64_t seed, int32_t level, bool singletons, int32_t *agg,
                  uint8_t *is_root, Arena &ar, int32_t **root_vertex, int32_t *rounds,
                  hipStream_t s) {
  if (order == 0 && n < (1 << 30))
    return aggregate_impl<uint32_t>(n, nnzG, grp, gcol, order, seed, level, singletons, agg,
                                    is_root, ar, root_vertex, rounds, s);
  return aggregate_impl<uint64_t>(n, nnzG, grp, gcol, order, seed, level, singletons, agg,
                                  is_root, ar, root_vertex, rounds, s);
}

// ---- Sprsfy (Sec. 2.5) --------------------------------------------------------------------
constexpr int32_t kSprsfyShort = 32;   // root rows up to this length: one thread per aggregate
constexpr int32_t kSprsfyLds = 4096;   // longer root rows (up to this): one block per aggregate
// ... unless the non-root members' rows hold more than this many entries in all: a thread
// scans them once per candidate, so such aggregates also take the block path
constexpr int32_t kSprsfyMemberWork = 128;
constexpr int32_t kSprsfySmall = 64;   // block path with LDS for root rows up to this length
// One thread per aggregate J with root r.  Candidates: aggregates reached by r's weak
// connections but by none of its strong ones, J excluded.  For a candidate c, a single strong
// connection from a non-root member of J into c is dropped with its transpose.  Decisions read
// "strong" as mask 1 or 2, so concurrent drops by other aggregates do not change them; the
// result depends neither on member order nor on the order in which aggregates are taken.
// Aggregates with a long root row or heavy members are listed for k_sprsfy_block: those with
// root rows up to kSprsfySmall in heavy[0, nc) (count nheavy[0]), those up to kSprsfyLds in
// heavy[nc, 2nc) (count nheavy[1]), longer ones for k_sprsfy_long in heavy[2nc, 3nc) (count
// nheavy[2]).
__global__ void k_sprsfy(int32_t nc, const int32_t *rp, const int32_t *col, uint8_t *mask,
                         const int32_t *agg, const int32_t *root_vertex, const int32_t *mrp,
                         const int32_t *mem, int32_t *heavy, int32_t *nheavy) {
  const int64_t J64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J64 >= nc) return;
  const int32_t J = (int32_t)J64;
  const int32_t r = root_vertex[J];
  const int32_t rb = rp[r], re = rp[r + 1];
  bool long_row = re - rb > kSprsfyShort;
  int32_t w = 0;  // entries in the non-root members' rows
  for (int32_t m = mrp[J]; m < mrp[J + 1] && !long_row; ++m) {
    const int32_t v = mem[m];
    if (v != r) w += rp[v + 1] - rp[v];
  }
  if (long_row || w > kSprsfyMemberWork) {
    // root rows up to kSprsfySmall: the small-LDS list; up to kSprsfyLds: the second list;
    // longer ones: the third
    const int which = re - rb > kSprsfyLds ? 2 : re - rb > kSprsfySmall ? 1 : 0;
    heavy[which * (int64_t)nc + atomicAdd(nheavy + which, 1)] = J;
    return;
  }
  for (int32_t k = rb; k < re; ++k) {
    const int32_t u0 = col[k];
    if (u0 == r || mask[k] != 0) continue;  // weak connections of the root only
    const int32_t c = agg[u0];
    if (c < 0 || c == J) continue;
    bool first = true, strong_reached = false;
    for (int32_t q = rb; q < re; ++q) {
      const int32_t uq = col[q];
      if (uq == r || agg[uq] != c) continue;
      const uint8_t mq = mask[q];
      if (mq == 1 || mq == 2) strong_reached = true;
      else if (q < k) first = false;  // an earlier weak connection already reached c
    }
    if (!first || strong_reached) continue;
    // count strong connections from non-root members of J into c
    int32_t count = 0, ev = -1, vv = -1;
    for (int32_t m = mrp[J]; m < mrp[J + 1] && count < 2; ++m) {
      const int32_t v = mem[m];
      if (v == r) continue;
      for (int32_t q = rp[v]; q < rp[v + 1]; ++q) {
        const int32_t u = col[q];
        if (u == v) continue;
        const uint8_t mq = mask[q];
        if ((mq == 1 || mq == 2) && agg[u] == c) {
          ++count;
          ev = q;
          vv = v;
        }
      }
    }
    if (count != 1) continue;
    mask[ev] = 2;
    const int32_t u = col[ev];
    int32_t lo = rp[u], hi = rp[u + 1] - 1;
    while (lo <= hi) {
      const int32_t mid = (lo + hi) >> 1;
      const int32_t cm = col[mid];
      if (cm == vv) {
        if (mask[mid] == 1) mask[mid] = 2;
        break;
      }
      if (cm < vv) lo = mid + 1;
      else hi = mid - 1;
    }
  }
}

// The aggregates k_sprsfy lists (a long root row or heavy members), one block each: the root
// row's (aggregate, strong) pairs are sorted in LDS; a candidate is an aggregate reached only
// through weak entries (not J, not unaggregated).  Strong entries of the non-root members are
// counted per candidate (binary search in the sorted candidate list); a count of 1 drops that
// entry and its transpose.  Same decisions as k_sprsfy.
__device__ inline void bitonic_u64_blk(uint64_t *a, int32_t L) {
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
template <int CAP>
__global__ __launch_bounds__(kBlock) void k_sprsfy_block(const int32_t *heavy,
                                                         const int32_t *rp,
                                                         const int32_t *col, uint8_t *mask,
                                                         const int32_t *agg,
                                                         const int32_t *root_vertex,
                                                         const int32_t *mrp,
                                                         const int32_t *mem) {
  __shared__ uint64_t pairs[CAP];
  __shared__ int32_t cand[CAP];
  __shared__ int32_t cnt[CAP];
  __shared__ int32_t edge[CAP];
  __shared__ int32_t s_nc;
  const int32_t J = heavy[blockIdx.x];
  const int32_t r = root_vertex[J];
  const int32_t rb = rp[r], re = rp[r + 1];
  const int32_t len = re - rb;
  if (len > CAP) return;  // never: k_sprsfy lists longer root rows for k_sprsfy_long
  int32_t L = 1;
  while (L < len) L <<= 1;
  // key = (aggregate + 1) << 1 | strong ; entries that cannot be candidates sort first as 0
  for (int32_t q = threadIdx.x; q < L; q += blockDim.x) {
    uint64_t key = ~0ull;
    if (q < len) {
      const int32_t k = rb + q;
      const int32_t u = col[k];
      const int32_t c = (u == r) ? -1 : agg[u];
      const uint8_t m = mask[k];
      const bool strong = (m == 1 || m == 2);
      key = (c < 0) ? 0ull : (((uint64_t)(c + 1) << 1) | (strong ? 1u : 0u));
    }
    pairs[q] = key;
  }
  if (threadIdx.x == 0) s_nc = 0;
  __syncthreads();
  bitonic_u64_blk(pairs, L);
  // run heads: first entry of each aggregate; candidate if no strong entry in its run
  for (int32_t q = threadIdx.x; q < len; q += blockDim.x) {
    const uint64_t x = pairs[q];
    if (x == 0ull || x == ~0ull) continue;
    const int32_t c = (int32_t)(x >> 1) - 1;
    const bool head = q == 0 || (pairs[q - 1] >> 1) != (x >> 1);
    if (!head) continue;
    int32_t t = q;
    bool strong = false;
    while (t < len && (pairs[t] >> 1) == (x >> 1)) strong |= (pairs[t++] & 1) != 0;
    if (!strong && c != J) {
      const int32_t slot = atomicAdd(&s_nc, 1);
      cand[slot] = c;
    }
  }
  __syncthreads();
  const int32_t ncand = s_nc;
  if (ncand == 0) return;  // block-uniform
  // sort the candidate list (small) for binary search
  for (int32_t q = threadIdx.x; q < L; q += blockDim.x)
    pairs[q] = q < ncand ? (uint64_t)(uint32_t)cand[q] : ~0ull;
  __syncthreads();
  bitonic_u64_blk(pairs, L);
  for (int32_t q = threadIdx.x; q < ncand; q += blockDim.x) {
    cand[q] = (int32_t)pairs[q];
    cnt[q] = 0;
    edge[q] = -1;
  }
  __syncthreads();
  // one wavefront per member (4 members at a time), lanes over the member's row
  for (int32_t mm = mrp[J] + (int32_t)(threadIdx.x >> 6); mm < mrp[J + 1]; mm += kBlock / 64) {
    const int32_t v = mem[mm];
    if (v == r) continue;
    for (int32_t k = rp[v] + (int32_t)(threadIdx.x & 63); k < rp[v + 1]; k += 64) {
      const int32_t u = col[k];
      if (u == v) continue;
      const uint8_t m = mask[k];
      if (!(m == 1 || m == 2)) continue;
      const int32_t c = agg[u];
      if (c < 0) continue;
      int32_t lo = 0, hi = ncand - 1;
      while (lo <= hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (cand[mid] == c) {
          atomicAdd(&cnt[mid], 1);
          edge[mid] = k;
          break;
        }
        if (cand[mid] < c) lo = mid + 1;
        else hi = mid - 1;
      }
    }
  }
  __syncthreads();
  for (int32_t q = threadIdx.x; q < ncand; q += blockDim.x) {
    if (cnt[q] != 1) continue;
    const int32_t ev = edge[q];
    mask[ev] = 2;
    const int32_t u = col[ev];
    // the row holding ev: search the members for the one whose row range contains it
    int32_t vv = -1;
    for (int32_t mm = mrp[J]; mm < mrp[J + 1]; ++mm) {
      const int32_t v = mem[mm];
      if (ev >= rp[v] && ev < rp[v + 1]) {
        vv = v;
        break;
      }
    }
    int32_t lo = rp[u], hi = rp[u + 1] - 1;
    while (lo <= hi) {
      const int32_t mid = (lo + hi) >> 1;
      const int32_t cm = col[mid];
      if (cm == vv) {
        if (mask[mid] == 1) mask[mid] = 2;
        break;
      }
      if (cm < vv) lo = mid + 1;
      else hi = mid - 1;
    }
  }
}

// Aggregates whose root row is longer than kSprsfyLds, one block each: k_sprsfy's decisions
// from global memory, the root row's entries shared out over the block's threads.  The thread
// holding a candidate's first weak entry decides that candidate (the others skip it as not
// first), so each candidate is decided once, as in k_sprsfy, for any row length.
__global__ __launch_bounds__(kBlock) void k_sprsfy_long(const int32_t *list, const int32_t *rp,
                                                        const int32_t *col, uint8_t *mask,
                                                        const int32_t *agg,
                                                        const int32_t *root_vertex,
                                                        const int32_t *mrp,
                                                        const int32_t *mem) {
  const int32_t J = list[blockIdx.x];
  const int32_t r = root_vertex[J];
  const int32_t rb = rp[r], re = rp[r + 1];
  for (int32_t k = rb + (int32_t)threadIdx.x; k < re; k += blockDim.x) {
    const int32_t u0 = col[k];
    if (u0 == r || mask[k] != 0) continue;  // weak connections of the root only
    const int32_t c = agg[u0];
    if (c < 0 || c == J) continue;
    bool first = true, strong_reached = false;
    for (int32_t q = rb; q < re && first && !strong_reached; ++q) {
      const int32_t uq = col[q];
      if (uq == r || agg[uq] != c) continue;
      const uint8_t mq = mask[q];
      if (mq == 1 || mq == 2) strong_reached = true;
      else if (q < k) first = false;  // an earlier weak connection already reached c
    }
    if (!first || strong_reached) continue;
    int32_t count = 0, ev = -1, vv = -1;
    for (int32_t m = mrp[J]; m < mrp[J + 1] && count < 2; ++m) {
      const int32_t v = mem[m];
      if (v == r) continue;
      for (int32_t q = rp[v]; q < rp[v + 1]; ++q) {
        const int32_t u = col[q];
        if (u == v) continue;
        const uint8_t mq = mask[q];
        if ((mq == 1 || mq == 2) && agg[u] == c) {
          ++count;
          ev = q;
          vv = v;
        }
      }
    }
    if (count != 1) continue;
    mask[ev] = 2;
    const int32_t u = col[ev];
    int32_t lo = rp[u], hi = rp[u + 1] - 1;
    while (lo <= hi) {
      const int32_t mid = (lo + hi) >> 1;
      const int32_t cm = col[mid];
      if (cm == vv) {
        if (mask[mid] == 1) mask[mid] = 2;
        break;
      }
      if (cm < vv) lo = mid + 1;
      else hi = mid - 1;
    }
  }
}

void sprsfy(int32_t n, const int32_t *rp, const int32_t *col, uint8_t *mask, const int32_t *agg,
            const int32_t *root_vertex, int32_t nc, hipStream_t s) {
  if (nc <= 0) return;
  Arena tmp;
  tmp.stream = s;
  int32_t *mrp, *mem;
  member_lists(n, agg, nc, false, tmp, &mrp, &mem, s);  // decisions ignore member order
  // words: heavy aggregates with root rows [0] up to kSprsfySmall, [1] up to kSprsfyLds,
  // [2] longer; heavy holds the three lists at offsets 0, nc and 2 nc
  int32_t *words = tmp.alloc<int32_t>(3);
  int32_t *heavy = tmp.alloc<int32_t>(3 * (int64_t)nc);
  fill_i32(words, 0, 3, s);
  k_sprsfy<<<grid_for(nc), kBlock, 0, s>>>(nc, rp, col, mask, agg, root_vertex, mrp, mem,
                                           heavy, words);
  SA_LAUNCH_CHECK();
  int32_t nh[3];
  readback(nh, words, sizeof(nh), s);
  if (nh[0] > 0)
    k_sprsfy_block<kSprsfySmall><<<(unsigned)nh[0], kBlock, 0, s>>>(
        heavy, rp, col, mask, agg, root_vertex, mrp, mem);
  if (nh[1] > 0)
    k_sprsfy_block<kSprsfyLds><<<(unsigned)nh[1], kBlock, 0, s>>>(
        heavy + nc, rp, col, mask, agg, root_vertex, mrp, mem);
  if (nh[2] > 0)
    k_sprsfy_long<<<(unsigned)nh[2], kBlock, 0, s>>>(heavy + 2 * (int64_t)nc, rp, col, mask,
                                                     agg, root_vertex, mrp, mem);
  SA_LAUNCH_CHECK();
}

// ---- filtered matrix (Sec. 1.1 plain lumping; Sec. 2.3 Algorithm 2) and its diagonal -----
// Kept entries per row (the diagonal and the strong entries), entry-parallel like k_strength.
__global__ __launch_bounds__(kBlock) void k_lump_count(int32_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const uint8_t *__restrict__ mask,
                                                       int32_t *__restrict__ cnt) {
  __shared__ int32_t s_rp[kBlock + 1];
  __shared__ int32_t s_cnt[kBlock];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kBlock;
  const int32_t nr = (int32_t)min<int64_t>(kBlock, (int64_t)n - r0);
  if (t < nr) s_rp[t] = rp[r0 + t];
  if (t == 0) s_rp[nr] = rp[r0 + nr];  // nr can be kBlock: no thread t == nr
  s_cnt[t] = 0;
  __syncthreads();
  const int32_t e0 = s_rp[0], e1 = s_rp[nr];
  for (int32_t e = e0 + t; e < e1; e += kBlock) {
    const uint8_t m = mask[e];
    if (m == 1 || m == 3) {  // strong, or the diagonal
      int32_t lo = 0, hi = nr - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_rp[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      atomicAdd(&s_cnt[lo], 1);
    }
  }
  __syncthreads();
  if (t < nr) cnt[r0 + t] = s_cnt[t];
}

// One row of the filtered matrix and its smoothing diagonal.  A's row i is read at
// col/val/mask[k - ko] for k in [b, e); the filtered row is written at acol/aval[w - wo] for
// w from o (its row pointer) on -- global arrays (offsets 0) or a block's LDS copies.
__device__ __forceinline__ void lump_row(int32_t i, int32_t b, int32_t e, const int32_t *col,
                                         const double *val, const uint8_t *mask, int32_t ko,
                                         int32_t o, int32_t *acol, double *aval, int32_t wo,
                                         bool offlmp, double tau, bool one_norm, double mult,
                                         double *__restrict__ invD, int32_t *__restrict__ err) {
  int32_t w = o, ds = o;
  double aii = 0.0, r = 0.0;
#pragma unroll 8
  for (int32_t k = b; k < e; ++k) {
    const int32_t j = col[k - ko];
    if (j == i) {
      aii = val[k - ko];
      ds = w;
      acol[w - wo] = j;
      aval[w - wo] = val[k - ko];
      ++w;
    } else if (mask[k - ko] == 1) {
      acol[w - wo] = j;
      aval[w - wo] = val[k - ko];
      ++w;
    } else {
      r += val[k - ko];
    }
  }
  const int32_t wend = w;
  if (!offlmp || r >= 0.0 || !(aii > 0.0)) {
    aval[ds - wo] = aii + r;
  } else {
    double kp = 0.0, km = 0.0;
    bool has_kp = false, has_km = false;
    for (int32_t t = o; t < wend; ++t) {
      if (t == ds) continue;
      const double v = aval[t - wo];
      if (v > 0.0) {
        kp += v;
        has_kp = true;
      } else if (v < 0.0) {
        km += v;
        has_km = true;
      }
    }
    if (-r <= kp) {
      const double delta = r / kp;
      for (int32_t t = o; t < wend; ++t)
        if (t != ds && aval[t - wo] > 0.0) aval[t - wo] = aval[t - wo] * (1.0 + delta);
    } else {
      double offsum = 0.0;
      for (int32_t k = b; k < e; ++k)
        if (col[k - ko] != i) offsum += fabs(val[k - ko]);
      const double T = tau * (offsum / aii);
      const double rhat = r + kp;
      if (!has_km) {
        if (has_kp && fabs(r + kp) / aii <= T) {
          const double delta = r / kp;
          for (int32_t t = o; t < wend; ++t)
            if (t != ds && aval[t - wo] > 0.0) aval[t - wo] = aval[t - wo] * (1.0 + delta);
        }
      } else {
        const double a = aii;
        const double c = -km - rhat;
        const double U = fmin(fabs(rhat), a);
        const double bnd = T * a - c;
        double rs = 0.0;
        bool feasible;
        if (T > 1.0) {
          const double ub = bnd / (T - 1.0);
          feasible = ub >= 0.0;
          if (feasible) rs = fmin(U, ub);
        } else if (T < 1.0) {
          const double lb = bnd / (T - 1.0);
          feasible = lb <= U;
          if (feasible) rs = U;
        } else {
          feasible = bnd >= 0.0;
          if (feasible) rs = U;
        }
        if (!feasible) rs = (c <= a) ? U : 0.0;
        const double delta = (rhat + rs) / km;
        for (int32_t t = o; t < wend; ++t) {
          if (t == ds) continue;
          const double v = aval[t - wo];
          if (v > 0.0) aval[t - wo] = 0.0;
          else if (v < 0.0) aval[t - wo] = v * (1.0 + delta);
        }
        aval[ds - wo] = a - rs;
      }
    }
  }
  double D;
  if (one_norm) {
    D = 0.0;
    for (int32_t t = o; t < wend; ++t) D += fabs(aval[t - wo]);
    if (D == 0.0) {
      D = 1.0;
    } else {
      double sum = 0.0;
      for (int32_t t = o; t < wend; ++t) sum += aval[t - wo];
      if (D < mult * sum) D = mult * sum;
    }
  } else {
    D = aval[ds - wo];
    if (D == 0.0) atomicOr(err, 8);
  }
  invD[i] = 1.0 / D;
}

// Block b owns rows [R b, R b + R) (R <= 256 chosen so that the rows' entries usually fit
// kLumpCap).  When they fit, the entries are staged in LDS by all 256 threads with coalesced
// loads, threads t < R build their rows there, and the filtered rows (one contiguous run of
// Abar) are written back with coalesced stores; otherwise thread t works on row R b + t in
// global memory directly.
constexpr int32_t kLumpCap = 2048;
template <int R>
__global__ __launch_bounds__(kBlock) void k_lump_fill(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const double *__restrict__ val, const uint8_t *__restrict__ mask,
    const int32_t *__restrict__ arp, int32_t *__restrict__ acol, double *__restrict__ aval,
    bool offlmp, double tau, bool one_norm, double mult, double *__restrict__ invD,
    int32_t *__restrict__ err) {
  __shared__ int32_t s_col[kLumpCap], s_acol[kLumpCap];
  __shared__ double s_val[kLumpCap], s_aval[kLumpCap];
  __shared__ uint8_t s_mask[kLumpCap];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int32_t nr = (int32_t)min<int64_t>(R, (int64_t)n - r0);
  const int32_t e0 = rp[r0], e1 = rp[r0 + nr];
  const int32_t a0 = arp[r0], a1 = arp[r0 + nr];
  const int32_t i = (int32_t)r0 + t;
  if (e1 - e0 <= kLumpCap) {  // block-uniform; the filtered rows are no longer than A's
    for (int32_t k = e0 + t; k < e1; k += kBlock) {
      s_col[k - e0] = col[k];
      s_val[k - e0] = val[k];
      s_mask[k - e0] = mask[k];
    }
    __syncthreads();
    if (t < nr)
      lump_row(i, rp[i], rp[i + 1], s_col, s_val, s_mask, e0, arp[i], s_acol, s_aval, a0,
               offlmp, tau, one_norm, mult, invD, err);
    __syncthreads();
    for (int32_t w = a0 + t; w < a1; w += kBlock) {
      acol[w] = s_acol[w - a0];
      aval[w] = s_aval[w - a0];
    }
  } else if (t < nr) {
    lump_row(i, rp[i], rp[i + 1], col, val, mask, 0, arp[i], acol, aval, 0, offlmp, tau,
             one_norm, mult, invD, err);
  }
}

__global__ __launch_bounds__(kW) void k_lump_count_w(int32_t n, const int32_t *rp,
                                                     const int32_t *col, const uint8_t *mask,
                                                     int32_t *cnt) {
  SA_WAVE_ROW_BEGIN(n)
  int32_t c = 0;
  for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += kW) c += (col[k] == i || mask[k] == 1);
  c = wave_sum_i32(c);
  if (lane == 0) cnt[i] = c;
}

// Same arithmetic as k_lump_fill, one wavefront per row: the kept entries are compacted in
// parallel; every floating-point sum (removed entries, kept positives/negatives, original
// off-diagonal magnitudes, the 1-norm and the row sum) runs sequentially through
// wave_seq_sum; the scalar decisions are taken identically by all lanes.
__global__ __launch_bounds__(kW) void k_lump_fill_w(int32_t n, const int32_t *rp,
                                                    const int32_t *col, const double *val,
                                                    const uint8_t *mask, const int32_t *arp,
                                                    int32_t *acol, double *aval, bool offlmp,
                                                    double tau, bool one_norm, double mult,
                                                    double *invD, int32_t *err) {
  __shared__ double lds[kW];
  SA_WAVE_ROW_BEGIN(n)
  const int32_t b = rp[i], e = rp[i + 1];
  const int32_t o = arp[i], oe = arp[i + 1];
  int32_t w = o;
  int32_t ds = o;
  double aii = 0.0;
  for (int32_t c = b; c < e; c += kW) {
    const int32_t k = c + lane;
    bool kept = false, isd = false;
    int32_t j = 0;
    double v = 0.0;
    if (k < e) {
      j = col[k];
      v = val[k];
      isd = (j == i);
      kept = isd || mask[k] == 1;
    }
    const unsigned long long bm = __ballot(kept);
    const int32_t pos = w + __popcll(bm & ((1ull << lane) - 1ull));
    if (kept) {
      acol[pos] = j;
      aval[pos] = v;
    }
    const unsigned long long dm = __ballot(isd);
    if (dm) {
      const int dl = __ffsll((long long)dm) - 1;
      ds = __shfl(pos, dl, 64);
      aii = __shfl(v, dl, 64);
    }
    w += __popcll(bm);
  }
  __syncthreads();
  const double r = wave_seq_sum(b, e, [&](int32_t k) {
    return (col[k] != i && mask[k] != 1) ? val[k] : 0.0;
  }, lds);
  if (!offlmp || r >= 0.0 || !(aii > 0.0)) {
    if (lane == 0) aval[ds] = aii + r;
  } else {
    const double kp = wave_seq_sum(o, oe, [&](int32_t t) {
      return (t != ds && aval[t] > 0.0) ? aval[t] : 0.0;
    }, lds);
    const double km = wave_seq_sum(o, oe, [&](int32_t t) {
      return (t != ds && aval[t] < 0.0) ? aval[t] : 0.0;
    }, lds);
    bool hp = false, hm = false;
    for (int32_t t = o + lane; t < oe; t += kW) {
      if (t == ds) continue;
      hp |= aval[t] > 0.0;
      hm |= aval[t] < 0.0;
    }
    const bool has_kp = wave_any(hp), has_km = wave_any(hm);
    __syncthreads();
    if (-r <= kp) {
      const double delta = r / kp;
      for (int32_t t = o + lane; t < oe; t += kW)
        if (t != ds && aval[t] > 0.0) aval[t] = aval[t] * (1.0 + delta);
    } else {
      const double offsum = wave_seq_sum(b, e, [&](int32_t k) {
        return col[k] != i ? fabs(val[k]) : 0.0;
      }, lds);
      const double T = tau * (offsum / aii);
      const double rhat = r + kp;
      if (!has_km) {
        if (has_kp && fabs(r + kp) / aii <= T) {
          const double delta = r / kp;
          for (int32_t t = o + lane; t < oe; t += kW)
            if (t != ds && aval[t] > 0.0) aval[t] = aval[t] * (1.0 + delta);
        }
      } else {
        const double a = aii;
        const double c = -km - rhat;
        const double U = fmin(fabs(rhat), a);
        const double bnd = T * a - c;
        double rs = 0.0;
        bool feasible;
        if (T > 1.0) {
          const double ub = bnd / (T - 1.0);
          feasible = ub >= 0.0;
          if (feasible) rs = fmin(U, ub);
        } else if (T < 1.0) {
          const double lb = bnd / (T - 1.0);
          feasible = lb <= U;
          if (feasible) rs = U;
        } else {
          feasible = bnd >= 0.0;
          if (feasible) rs = U;
        }
        if (!feasible) rs = (c <= a) ? U : 0.0;
        const double delta = (rhat + rs) / km;
        for (int32_t t = o + lane; t < oe; t += kW) {
          if (t == ds) continue;
          const double v = aval[t];
          if (v > 0.0) aval[t] = 0.0;
          else if (v < 0.0) aval[t] = v * (1.0 + delta);
        }
        __syncthreads();
        if (lane == 0) aval[ds] = a - rs;
      }
    }
  }
  __syncthreads();
  double D;
  if (one_norm) {
    D = wave_seq_sum(o, oe, [&](int32_t t) { return fabs(aval[t]); }, lds);
    if (D == 0.0) {
      D = 1.0;
    } else {
      const double sum = wave_seq_sum(o, oe, [&](int32_t t) { return aval[t]; }, lds);
      if (D < mult * sum) D = mult * sum;
    }
  } else {
    D = aval[ds];
    if (D == 0.0 && lane == 0) atomicOr(err, 8);
  }
  if (lane == 0) invD[i] = 1.0 / D;
}

int64_t lump(int32_t n, int64_t nnz_a, const int32_t *rp, const int32_t *col, const double *val,
             const uint8_t *mask, bool offlmp, double tau, bool one_norm, double mult,
             bool wave, Arena &ar, Csr &abar, double *invD, int32_t *err, hipStream_t s) {
  int32_t *cnt = (int32_t *)dev_alloc(sizeof(int32_t) * (n + 1), s);
  if (wave) k_lump_count_w<<<(unsigned)n, kW, 0, s>>>(n, rp, col, mask, cnt);
  else k_lump_count<<<grid_for(n), kBlock, 0, s>>>(n, rp, col, mask, cnt);
  SA_LAUNCH_CHECK();
  abar.n = abar.ncols = n;
  abar.rp = ar.alloc<int32_t>(n + 1);
  exclusive_scan_i32(cnt, abar.rp, n, s);
  dev_free(cnt, s);
  abar.nnz = read1(abar.rp + n, s);
  abar.col = ar.alloc<int32_t>(abar.nnz);
  abar.val = ar.alloc<double>(abar.nnz);
  if (wave)
    k_lump_fill_w<<<(unsigned)n, kW, 0, s>>>(n, rp, col, val, mask, abar.rp, abar.col, abar.val,
                                             offlmp, tau, one_norm, mult, invD, err);
  else if (nnz_a <= 7 * (int64_t)n)
    k_lump_fill<256><<<(unsigned)ceil_div(n, 256), kBlock, 0, s>>>(
        n, rp, col, val, mask, abar.rp, abar.col, abar.val, offlmp, tau, one_norm, mult, invD,
        err);
  else if (nnz_a <= 15 * (int64_t)n)
    k_lump_fill<128><<<(unsigned)ceil_div(n, 128), kBlock, 0, s>>>(
        n, rp, col, val, mask, abar.rp, abar.col, abar.val, offlmp, tau, one_norm, mult, invD,
        err);
  else
    k_lump_fill<64><<<(unsigned)ceil_div(n, 64), kBlock, 0, s>>>(
        n, rp, col, val, mask, abar.rp, abar.col, abar.val, offlmp, tau, one_norm, mult, invD,
        err);
  SA_LAUNCH_CHECK();
  return abar.nnz;
}

// ---- power method (Sec. 1.1 damping; Sec. 3.1 ten sweeps) --------------------------------
__global__ void k_power_init(int32_t n, uint64_t seed, int32_t level, int32_t stream,
                             double *x) {
  SA_ROW_KERNEL_BEGIN(n)
  const uint64_t z = splitmix64_dev(seed, stream_key_dev(stream, level, i));
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  x[i] = 2.0 * u - 1.0;
}
// x = y / 2^ilogb(m) with m = max |y_i|: every block reduces the kMaxSlots maxima that the
// SpMV left (bit patterns of non-negative doubles, monotone), and block 0 clears the other
// slot set, which the next iteration's SpMV fills.  A zero or non-finite maximum marks the
// iteration dead.
__global__ __launch_bounds__(kBlock) void k_normalize(int32_t n, const double *y,
                                                      const unsigned long long *slots,
                                                      unsigned long long *next, double *x,
                                                      int32_t *dead) {
  static_assert(kMaxSlots == kBlock, "one slot per thread");
  __shared__ unsigned long long wm[kBlock / 64];
  unsigned long long m = slots[threadIdx.x];
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  if (blockIdx.x == 0) next[threadIdx.x] = 0ull;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q) m = wm[q] > m ? wm[q] : m;
  SA_ROW_KERNEL_BEGIN(n)
  const double mv = __longlong_as_double((long long)m);
  if (!(mv > 0.0) || !isfinite(mv)) {
    if (i == 0) *dead = 1;
    return;
  }
  x[i] = ldexp(y[i], -ilogb(mv));
}
__global__ void k_rayleigh(const double *xy, const double *xx, const int32_t *dead,
                           double *lam) {
  *lam = (*dead) ? 0.0 : (*xy / *xx);
}

void power_method(const Csr &M, const double *invD, int32_t iters, uint64_t seed, int32_t level,
                  int32_t stream_id, double *lam, hipStream_t s) {
  const int32_t n = M.n;
  Arena tmp;
  tmp.stream = s;
  double *x = tmp.alloc<double>(n);
  double *y = tmp.alloc<double>(n);
  double *ws = tmp.alloc<double>(dot_ws_size(n));
  double *sc = tmp.alloc<double>(4);
  // two sets of kMaxSlots maxima (iteration t fills set t mod 2), then the dead flag
  unsigned long long *mx = tmp.alloc<unsigned long long>(2 * kMaxSlots + 1);
  int32_t *dead = (int32_t *)(mx + 2 * kMaxSlots);
  fill_i32((int32_t *)mx, 0, 2 * (2 * kMaxSlots + 1), s);
  k_power_init<<<grid_for(n), kBlock, 0, s>>>(n, seed, level, stream_id, x);
  SA_LAUNCH_CHECK();
  SpmvArgs<double> a = spmv_args<double>(M, M.val, x);
  a.plain = true;  // the estimate decides the hierarchy: every row in sequential order
  for (int32_t t = 1; t <= iters; ++t) {
    unsigned long long *cur = mx + (t & 1) * kMaxSlots, *nxt = mx + ((t + 1) & 1) * kMaxSlots;
    if (t == iters) spmv_scale<double>(a, invD, y, s);
    else spmv_scale_max<double>(a, invD, y, cur, s);
    if (t == iters) {
      dot_f64(x, y, n, sc + 0, ws, s);
      dot_f64(x, x, n, sc + 1, ws, s);
      k_rayleigh<<<1, 1, 0, s>>>(sc + 0, sc + 1, dead, lam);
      SA_LAUNCH_CHECK();
      break;
    }
    k_normalize<<<grid_for(n), kBlock, 0, s>>>(n, y, cur, nxt, x, dead);
    SA_LAUNCH_CHECK();
  }
}

__global__ void k_damping(double *lam, double *omega, bool unit, int32_t *err) {
  if (unit) *lam = 1.0;
  const double l = *lam;
  if (!(l > 0.0) || !isfinite(l)) atomicOr(err, 16);
  *omega = 4.0 / (3.0 * l);
}
void damping(double *lam, double *omega, bool unit, int32_t *err, hipStream_t s) {
  k_damping<<<1, 1, 0, s>>>(lam, omega, unit, err);
  SA_LAUNCH_CHECK();
}

// ---- prolongator smoothing (Sec. 1.1) -------------------------------------------------------
// Row i: for each aggregate J reached by the filtered row (ascending J), acc = sum of the
// entries with agg(k) = J in ascending k from 0; P_iJ = [J == agg_i] - (omega invD_i) acc.
// Rows of at most kPRegs entries keep their aggregates (and values) in registers, loaded as
// independent loads up front; longer rows re-read them per distinct aggregate.
constexpr int kPRegs = 16;
// Rows of up to R entries: the entries' aggregates (and values) loaded once, in one batch,
// and the distinct aggregates counted, or summed in ascending aggregate order, in registers.
template <int R>
__device__ __forceinline__ int32_t p_count_regs(int32_t b, int32_t e,
                                                const int32_t *__restrict__ col,
                                                const int32_t *__restrict__ agg) {
  int32_t a[R];
#pragma unroll
  for (int q = 0; q < R; ++q) a[q] = (b + q < e) ? col[min(b + q, e - 1)] : -1;
#pragma unroll
  for (int q = 0; q < R; ++q) a[q] = (a[q] >= 0) ? agg[a[q]] : -1;
  // distinct aggregates = entries whose aggregate does not occur earlier in the row
  int32_t c = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    bool first = a[q] >= 0;
#pragma unroll
    for (int r = 0; r < q; ++r) first = first && (a[r] != a[q]);
    c += first;
  }
  return c;
}
template <int R>
__device__ __forceinline__ void p_fill_regs(int32_t rb, int32_t re,
                                            const int32_t *__restrict__ col,
                                            const double *__restrict__ val,
                                            const int32_t *__restrict__ agg, int32_t ai, double t,
                                            int32_t w, int32_t *__restrict__ pcol,
                                            double *__restrict__ pval) {
  int32_t a[R];
  double v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int32_t k = min(rb + q, re - 1);
    a[q] = (rb + q < re) ? col[k] : -1;
    v[q] = (rb + q < re) ? val[k] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) a[q] = (a[q] >= 0) ? agg[a[q]] : -1;
  // aggregates in ascending order; each sums its entries in ascending position from 0
  int32_t prev = -1;
  for (;;) {
    int32_t J = INT_MAX;
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (a[q] > prev && a[q] < J) J = a[q];
    if (J == INT_MAX) break;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (a[q] == J) acc += v[q];
    pcol[w] = J;
    pval[w] = ((J == ai) ? 1.0 : 0.0) - t * acc;
    ++w;
    prev = J;
  }
}

__global__ void k_P_count(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *agg,
                          int32_t *cnt) {
  SA_ROW_KERNEL_BEGIN(n)
  const int32_t b = rp[i], e = rp[i + 1];
  if (e <= b) {
    cnt[i] = 0;
    return;
  }
  if (e - b <= kPRegs) {
    cnt[i] = p_count_regs<kPRegs>(b, e, col, agg);
    return;
  }
  if (e - b <= 2 * kPRegs) {
    cnt[i] = p_count_regs<2 * kPRegs>(b, e, col, agg);
    return;
  }
  int32_t prev = -1, c = 0;
  for (;;) {
    int32_t J = INT_MAX;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t a = agg[col[k]];
      if (a > prev && a < J) J = a;
    }
    if (J == INT_MAX) break;
    ++c;
    prev = J;
  }
  cnt[i] = c;
}
__global__ void k_P_fill(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                         const double *invD, const int32_t *agg, const double *omega,
                         const int32_t *prp, int32_t *pcol, double *pval) {
  SA_ROW_KERNEL_BEGIN(n)
  const double t = (*omega) * invD[i];
  const int32_t ai = agg[i];
  const int32_t rb = rp[i], re = rp[i + 1];
  if (re <= rb) return;  // an empty row has no prolongator entries
  if (re - rb <= kPRegs) {
    p_fill_regs<kPRegs>(rb, re, col, val, agg, ai, t, prp[i], pcol, pval);
    return;
  }
  if (re - rb <= 2 * kPRegs) {
    p_fill_regs<2 * kPRegs>(rb, re, col, val, agg, ai, t, prp[i], pcol, pval);
    return;
  }
  int32_t prev = -1, w = prp[i];
  for (;;) {
    int32_t J = INT_MAX;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t a = agg[col[k]];
      if (a > prev && a < J) J = a;
    }
    if (J == INT_MAX) break;
    double acc = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (agg[col[k]] == J) acc += val[k];
    pcol[w] = J;
    pval[w] = ((J == ai) ? 1.0 : 0.0) - t * acc;
    ++w;
    prev = J;
  }
}
// Long rows (the dense coarse levels): the per-aggregate sums of a row of Abar are the row of
// Abar T, T the 0/1 aggregate matrix (T_kJ = 1 iff agg_k = J): every product is A_ik * 1 =
// A_ik exactly and the SpGEMM adds them in ascending k from 0, the order of k_P_fill.  Then
// P_iJ = [J = agg_i] - t_i (Abar T)_iJ in place.
__global__ void k_agg_matrix(int32_t n, const int32_t *agg, const int32_t *trp, int32_t *tcol,
                             double *tval) {
  SA_ROW_KERNEL_BEGIN(n)
  if (agg[i] >= 0) {
    tcol[trp[i]] = agg[i];
    tval[trp[i]] = 1.0;
  }
}
__global__ void k_flag_aggregated(int32_t n, const int32_t *agg, int32_t *f) {
  SA_ROW_KERNEL_BEGIN(n)
  f[i] = agg[i] >= 0 ? 1 : 0;
}
__global__ void k_P_from_sums(int32_t n, const int32_t *prp, const int32_t *pcol, double *pval,
                              const double *invD, const int32_t *agg, const double *omega) {
  SA_ROW_KERNEL_BEGIN(n)
  const double t = (*omega) * invD[i];
  const int32_t ai = agg[i];
  for (int32_t e = prp[i]; e < prp[i + 1]; ++e)
    pval[e] = ((pcol[e] == ai) ? 1.0 : 0.0) - t * pval[e];
}

int64_t prolongator(const Csr &abar, const double *invD, const int32_t *agg, int32_t nc,
                    const double *omega, Arena &ar, Csr &P, hipStream_t s, bool long_rows) {
  const int32_t n = abar.n;
  if (long_rows && n > 0) {
    Arena tmp;
    tmp.stream = s;
    int32_t *f = tmp.alloc<int32_t>(n + 1);
    k_flag_aggregated<<<grid_for(n), kBlock, 0, s>>>(n, agg, f);
    SA_LAUNCH_CHECK();
    Csr T;
    T.n = n;
    T.ncols = nc;
    T.rp = tmp.alloc<int32_t>(n + 1);
    exclusive_scan_i32(f, T.rp, n, s);
    T.nnz = read1(T.rp + n, s);
    T.col = tmp.alloc<int32_t>(T.nnz > 0 ? T.nnz : 1);
    T.val = tmp.alloc<double>(T.nnz > 0 ? T.nnz : 1);
    k_agg_matrix<<<grid_for(n), kBlock, 0, s>>>(n, agg, T.rp, T.col, T.val);
    SA_LAUNCH_CHECK();
    spgemm(abar, T, ar, P, s);
    k_P_from_sums<<<grid_for(n), kBlock, 0, s>>>(n, P.rp, P.col, P.val, invD, agg, omega);
    SA_LAUNCH_CHECK();
    return P.nnz;
  }
  int32_t *cnt = (int32_t *)dev_alloc(sizeof(int32_t) * (n + 1), s);
  k_P_count<<<grid_for(n), kBlock, 0, s>>>(n, abar.rp, abar.col, agg, cnt);
  SA_LAUNCH_CHECK();
  P.n = n;
  P.ncols = nc;
  P.rp = ar.alloc<int32_t>(n + 1);
  exclusive_scan_i32(cnt, P.rp, n, s);
  dev_free(cnt, s);
  P.nnz = read1(P.rp + n, s);
  P.col = ar.alloc<int32_t>(P.nnz);
  P.val = ar.alloc<double>(P.nnz);
  k_P_fill<<<grid_for(n), kBlock, 0, s>>>(n, abar.rp, abar.col, abar.val, invD, agg, omega, P.rp,
                                          P.col, P.val);
  SA_LAUNCH_CHECK();
  return P.nnz;
}

// ---- Cnstrnt (Sec. 2.4, Algorithm 3, with the loop run while any bound is violated) ------
__global__ void k_cnstrnt(int32_t n, const int32_t *rp, const int32_t *col, double *v,
                          const int32_t *agg, uint8_t *inw) {
  SA_ROW_KERNEL_BEGIN(n)
  const int32_t b = rp[i], e = rp[i + 1];
  bool viol = false;
  for (int32_t k = b; k < e; ++k)
    if (v[k] < 0.0 || v[k] > 1.0) viol = true;
  if (!viol) return;
  int32_t cnt = 0;
  double sum = 0.0;
  for (int32_t k = b; k < e; ++k) {
    inw[k] = v[k] != 0.0;
    if (inw[k]) {
      ++cnt;
      sum += v[k];
    }
  }
  const int32_t ai = agg[i];
  bool tent = false;
  if (sum < 0.0 || sum > (double)cnt) {
    tent = true;
  } else if (sum == 0.0) {
    for (int32_t k = b; k < e; ++k) v[k] = 0.0;
    return;
  } else {
    while (cnt > 0) {
      int32_t kmin = -1, kmax = -1;
      for (int32_t k = b; k < e; ++k) {
        if (!inw[k]) continue;
        if (kmin < 0 || v[k] < v[kmin]) kmin = k;
        if (kmax < 0 || v[k] > v[kmax]) kmax = k;
      }
      if (!(v[kmin] < 0.0 || v[kmax] > 1.0)) break;
      double delta = 0.0;
      if (v[kmin] < 0.0) {
        delta += v[kmin];
        v[kmin] = 0.0;
        inw[kmin] = 0;
        --cnt;
      }
      if (v[kmax] > 1.0) {
        delta += v[kmax] - 1.0;
        v[kmax] = 1.0;
        inw[kmax] = 0;
        --cnt;
      }
      if (cnt == 0) {
        if (delta != 0.0) tent = true;
        break;
      }
      const double q = delta / (double)cnt;
      for (int32_t k = b; k < e; ++k)
        if (inw[k]) v[k] += q;
    }
  }
  if (tent)
    for (int32_t k = b; k < e; ++k) v[k] = (col[k] == ai) ? 1.0 : 0.0;
}
void cnstrnt(const Csr &P, const int32_t *agg, hipStream_t s) {
  if (P.n <= 0) return;
  uint8_t *inw = (uint8_t *)dev_alloc(P.nnz > 0 ? P.nnz : 1, s);
  k_cnstrnt<<<grid_for(P.n), kBlock, 0, s>>>(P.n, P.rp, P.col, P.val, agg, inw);
  SA_LAUNCH_CHECK();
  dev_free(inw, s);
}

__global__ void k_scale_rows(int32_t n, const int32_t *rp, double *val, const double *B) {
  SA_ROW_KERNEL_BEGIN(n)
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) val[k] = B[i] * val[k];
}
void scale_rows(const Csr &P, const double *B, hipStream_t s) {
  if (P.n <= 0) return;
  k_scale_rows<<<grid_for(P.n), kBlock, 0, s>>>(P.n, P.rp, P.val, B);
  SA_LAUNCH_CHECK();
}

__global__ void k_scale_sym(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                            const double *B, double *out) {
  SA_ROW_KERNEL_BEGIN(n)
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) out[k] = (B[i] * val[k]) * B[col[k]];
}
void scale_sym(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
               const double *B, double *out, hipStream_t s) {
  if (n <= 0) return;
  k_scale_sym<<<grid_for(n), kBlock, 0, s>>>(n, rp, col, val, B, out);
  SA_LAUNCH_CHECK();
}


// ---- per-row sort by column --------------------------------------------------------------
// Rows of up to kSortShort entries: a register sorting network in one thread (the keys of a
// row are distinct in every caller).  Longer rows: one block per
// row, bitonic sort in LDS (kSortLds entries) or, beyond that, in a global scratch region
// sized for the row.  Keys within a row are distinct, so the order is unique.
constexpr int32_t kSortShort = 32;
constexpr int32_t kSortLds = 4096;

__device__ inline void wave_append(bool pred, int32_t *counter, int32_t *list, int32_t value) {
  const unsigned long long m = __ballot(pred);
  if (!m) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader, 64);
  if (pred) list[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

// Sorts L <= N (key, value) pairs with distinct keys in registers: a bitonic network of width
// N over the pairs padded with INT_MAX keys, all indices static so nothing leaves registers.
template <int N>
__device__ __forceinline__ void sort_regs(int32_t *c, double *v, int32_t L) {
  int32_t kk[N];
  double vv[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    kk[q] = q < L ? c[q] : INT_MAX;
    vv[q] = (v && q < L) ? v[q] : 0.0;
  }
#pragma unroll
  for (int k = 2; k <= N; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const int l = q ^ j;
        if (l > q) {
          const bool up = (q & k) == 0;
          if ((kk[q] > kk[l]) == up) {
            const int32_t tk = kk[q];
            kk[q] = kk[l];
            kk[l] = tk;
            const double tv = vv[q];
            vv[q] = vv[l];
            vv[l] = tv;
          }
        }
      }
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (q < L) {
      c[q] = kk[q];
      if (v) v[q] = vv[q];
    }
}

__global__ void k_sort_short(int32_t n, const int32_t *rp, int32_t *c, double *v,
                             int32_t *nlong, int32_t *longrows) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i64 < n;
  const int32_t i = live ? (int32_t)i64 : 0;
  const int32_t b = live ? rp[i] : 0, e = live ? rp[i + 1] : 0;
  const bool is_long = live && (e - b > kSortShort);
  wave_append(is_long, nlong, longrows, i);
  if (!live || is_long) return;
  const int32_t L = e - b;
  if (L <= 1) return;
  if (L <= 8) sort_regs<8>(c + b, v ? v + b : nullptr, L);
  else if (L <= 16) sort_regs<16>(c + b, v ? v + b : nullptr, L);
  else sort_regs<32>(c + b, v ? v + b : nullptr, L);
}

__device__ inline void bitonic_kv_any(int32_t *k, double *v, int32_t L) {
  for (int32_t kk = 2; kk <= L; kk <<= 1) {
    for (int32_t j = kk >> 1; j > 0; j >>= 1) {
      for (int32_t idx = threadIdx.x; idx < L; idx += blockDim.x) {
        const int32_t ixj = idx ^ j;
        if (ixj > idx) {
          const int32_t x = k[idx], y = k[ixj];
          const bool up = (idx & kk) == 0;
          if ((x > y) == up) {
            k[idx] = y;
            k[ixj] = x;
            if (v) {
              const double t = v[idx];
              v[idx] = v[ixj];
              v[ixj] = t;
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// One block per long row; rows longer than kSortLds use gk/gv at goff[slot].
__global__ __launch_bounds__(kBlock) void k_sort_long(const int32_t *rows, int32_t nrows,
                                                      const int32_t *rp, int32_t *c, double *v,
                                                      int32_t *gk, double *gv,
                                                      const int64_t *goff) {
  __shared__ int32_t sk[kSortLds];
  __shared__ double sv[kSortLds];
  const int32_t slot = blockIdx.x;
  if (slot >= nrows) return;
  const int32_t i = rows[slot];
  const int32_t b = rp[i], len = rp[i + 1] - b;
  int32_t L = 1;
  while (L < len) L <<= 1;
  int32_t *kk;
  double *vv;
  if (L <= kSortLds) {
    kk = sk;
    vv = v ? sv : nullptr;
  } else {
    kk = gk + goff[slot];
    vv = v ? gv + goff[slot] : nullptr;
  }
  for (int32_t q = threadIdx.x; q < L; q += blockDim.x) {
    kk[q] = q < len ? c[b + q] : INT_MAX;
    if (vv) vv[q] = q < len ? v[b + q] : 0.0;
  }
  __syncthreads();
  bitonic_kv_any(kk, vv, L);
  for (int32_t q = threadIdx.x; q < len; q += blockDim.x) {
    c[b + q] = kk[q];
    if (v) v[b + q] = vv[q];
  }
}

__global__ void k_sort_caps(int32_t nrows, const int32_t *rows, const int32_t *rp,
                            int64_t *caps) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const int32_t i = rows[t];
  const int32_t len = rp[i + 1] - rp[i];
  int64_t L = 1;
  while (L < len) L <<= 1;
  caps[t] = (L <= kSortLds) ? 0 : L;
}

void sort_rows(int32_t n, const int32_t *rp, int32_t *col, double *val, hipStream_t s) {
  if (n <= 0) return;
  Arena tmp;
  tmp.stream = s;
  int32_t *nlong = tmp.alloc<int32_t>(1);
  int32_t *rows = tmp.alloc<int32_t>(n);
  fill_i32(nlong, 0, 1, s);
  k_sort_short<<<grid_for(n), kBlock, 0, s>>>(n, rp, col, val, nlong, rows);
  SA_LAUNCH_CHECK();
  const int32_t nl = read1(nlong, s);
  if (nl == 0) return;
  int64_t *caps = tmp.alloc<int64_t>(nl + 1);
  int64_t *goff = tmp.alloc<int64_t>(nl + 1);
  k_sort_caps<<<grid_for(nl), kBlock, 0, s>>>(nl, rows, rp, caps);
  SA_LAUNCH_CHECK();
  exclusive_scan_i64(caps, goff, nl, s);
  const int64_t gtot = read1(goff + nl, s);
  int32_t *gk = tmp.alloc<int32_t>(gtot > 0 ? gtot : 1);
  double *gv = tmp.alloc<double>(gtot > 0 ? gtot : 1);
  k_sort_long<<<(unsigned)nl, kBlock, 0, s>>>(rows, nl, rp, col, val, gk, gv, goff);
  SA_LAUNCH_CHECK();
}

// ---- transpose with values ---------------------------------------------------------------
__global__ void k_count_cols(int64_t nnz, const int32_t *col, int32_t *cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[col[e]], 1);
}
__global__ void k_scatter_tv(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                             int32_t *pos, int32_t *tcol, double *tval) {
  SA_ROW_KERNEL_BEGIN(n)
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const int32_t p = atomicAdd(&pos[col[k]], 1);
    tcol[p] = i;
    tval[p] = val[k];
  }
}
void transpose(const Csr &P, Arena &ar, Csr &R, hipStream_t s) {
  const int32_t m = P.ncols;
  int32_t *cnt = (int32_t *)dev_alloc(sizeof(int32_t) * (m + 1), s);
  fill_i32(cnt, 0, m + 1, s);
  if (P.nnz > 0) {
    k_count_cols<<<grid_for(P.nnz), kBlock, 0, s>>>(P.nnz, P.col, cnt);
    SA_LAUNCH_CHECK();
  }
  R.n = m;
  R.ncols = P.n;
  R.nnz = P.nnz;
  R.rp = ar.alloc<int32_t>(m + 1);
  exclusive_scan_i32(cnt, R.rp, m, s);
  SA_HIP(hipMemcpyAsync(cnt, R.rp, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToDevice, s));
  R.col = ar.alloc<int32_t>(P.nnz);
  R.val = ar.alloc<double>(P.nnz);
  if (P.n > 0) {
    k_scatter_tv<<<grid_for(P.n), kBlock, 0, s>>>(P.n, P.rp, P.col, P.val, cnt, R.col, R.val);
    SA_LAUNCH_CHECK();
  }
  sort_rows(m, R.rp, R.col, R.val, s);
  dev_free(cnt, s);
}

__global__ void k_inv_diag(int32_t n, const double *d, double *inv, int32_t *err) {
  SA_ROW_KERNEL_BEGIN(n)
  if (!(d[i] > 0.0)) atomicOr(err, 32);
  inv[i] = 1.0 / d[i];
}
void inv_diag(int32_t n, const double *dval, double *invD, int32_t *err, hipStream_t s) {
  if (n <= 0) return;
  k_inv_diag<<<grid_for(n), kBlock, 0, s>>>(n, dval, invD, err);
  SA_LAUNCH_CHECK();
}

}  // namespace sa
