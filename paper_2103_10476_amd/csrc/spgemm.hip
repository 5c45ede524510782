// Sparse matrix-matrix product C = X*Y for the Galerkin operator (Sec. 1.1), in Gustavson
// order: every output entry C_ij accumulates X_ik*Y_kj over the row's entries k in ascending
// order, from 0.  No floating-point atomics: each output row is expanded into its products in
// that order, stably sorted by output column, and every run of equal columns is summed by one
// lane in order.  Output rows are sorted; cancellations stay stored.
//
// Rows are binned by their product count T:
//   T <= 64      one wavefront per row: one product per lane, rank sort in LDS;
//   T > 64       one 256-thread block per row: chunks of 1024 products, bitonic sort of
//                (column, position) keys in LDS; a single chunk is reduced and written
//                directly, longer rows accumulate chunk by chunk into an LDS hash table
//                (same order per entry), which is sorted by column at the end;
//   hash > 1/2   rows whose distinct columns overflow the LDS table are redone with a table
//                in global memory sized for the row.
// Results go to per-row slots at the row's product offset (room for T >= distinct entries)
// and are compacted into CSR afterwards.
#include "kernels.hpp"

namespace sa {

constexpr int kWave = 64;
constexpr int kChunk = 1024;  // products per block-level chunk
constexpr int kHash = 4096;   // LDS hash capacity (entries)

__global__ void k_count_products(int32_t m, const int32_t *xrp, const int32_t *xcol,
                                 const int32_t *yrp, int64_t *cnt, int32_t *xpref) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= m) return;
  const int32_t i = (int32_t)i64;
  int64_t t = 0;
  for (int32_t e = xrp[i]; e < xrp[i + 1]; ++e) {
    xpref[e] = (int32_t)t;  // products before entry e within the row (T < 2^31 checked)
    const int32_t k = xcol[e];
    t += yrp[k + 1] - yrp[k];
  }
  cnt[i] = t;
}

__global__ void k_bin_rows(int32_t m, const int64_t *poff, int32_t *small, int32_t *big,
                           int32_t *counters) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= m) return;
  const int32_t i = (int32_t)i64;
  const int64_t T = poff[i + 1] - poff[i];
  if (T <= kWave) small[atomicAdd(&counters[0], 1)] = i;
  else big[atomicAdd(&counters[1], 1)] = i;
}

// ---- one wavefront per row (T <= 64) ------------------------------------------------------
__global__ __launch_bounds__(kWave) void k_esc_wave(
    const int32_t *rows, int32_t nrows, const int32_t *xrp, const int32_t *xcol,
    const double *xval, const int32_t *yrp, const int32_t *ycol, const double *yval,
    const int64_t *poff, int32_t *ocol, double *oval, int32_t *ucnt) {
  __shared__ int32_t keys[kWave];
  __shared__ double vals[kWave];
  __shared__ int32_t skeys[kWave];
  __shared__ double svals[kWave];
  const int lane = threadIdx.x;
  if ((int32_t)blockIdx.x >= nrows) return;  // block-uniform
  const int32_t i = rows[blockIdx.x];
  const int64_t base = poff[i];
  const int32_t T = (int32_t)(poff[i + 1] - base);
  // expansion in Gustavson order: position = products of earlier X entries + offset in Y row
  int32_t filled = 0;
  for (int32_t g = xrp[i]; g < xrp[i + 1]; g += kWave) {
    const int32_t e = g + lane;
    int32_t len = 0, ys = 0;
    double a = 0.0;
    if (e < xrp[i + 1]) {
      const int32_t k = xcol[e];
      a = xval[e];
      ys = yrp[k];
      len = yrp[k + 1] - ys;
    }
    // inclusive wave scan of len
    int32_t incl = len;
    for (int off = 1; off < kWave; off <<= 1) {
      const int32_t v = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += v;
    }
    const int32_t excl = incl - len;
    const int32_t tot = __shfl(incl, kWave - 1, kWave);
    for (int32_t t = 0; t < len; ++t) {
      const int32_t p = filled + excl + t;
      keys[p] = ycol[ys + t];
      vals[p] = a * yval[ys + t];
    }
    filled += tot;
  }
  __syncthreads();
  int32_t key = 0;
  double v = 0.0;
  if (lane < T) {
    key = keys[lane];
    v = vals[lane];
    int32_t rank = 0;
    for (int32_t q = 0; q < T; ++q) {
      const int32_t kq = keys[q];
      rank += (kq < key) || (kq == key && q < lane);
    }
    skeys[rank] = key;
    svals[rank] = v;
  }
  __syncthreads();
  bool head = false;
  double sum = 0.0;
  if (lane < T) {
    key = skeys[lane];
    head = (lane == 0) || (skeys[lane - 1] != key);
    if (head)
      for (int32_t r = lane; r < T && skeys[r] == key; ++r) sum += svals[r];
  }
  const unsigned long long hm = __ballot(head);
  const int32_t idx = __popcll(hm & ((1ull << lane) - 1ull));
  if (head) {
    ocol[base + idx] = key;
    oval[base + idx] = sum;
  }
  if (lane == 0) ucnt[i] = __popcll(hm);
}

// ---- one block per row (T > 64) -----------------------------------------------------------
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

// Sorts (key, value) pairs by key as unsigned (empty slots hold -1 and go last).
__device__ inline void bitonic_kv(int32_t *k, double *v, int32_t L) {
  for (int32_t kk = 2; kk <= L; kk <<= 1) {
    for (int32_t j = kk >> 1; j > 0; j >>= 1) {
      for (int32_t idx = threadIdx.x; idx < L; idx += blockDim.x) {
        const int32_t ixj = idx ^ j;
        if (ixj > idx) {
          const uint32_t x = (uint32_t)k[idx], y = (uint32_t)k[ixj];
          const bool up = (idx & kk) == 0;
          if ((x > y) == up) {
            k[idx] = (int32_t)y;
            k[ixj] = (int32_t)x;
            const double t = v[idx];
            v[idx] = v[ixj];
            v[ixj] = t;
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

// GLOBAL = false: hash table in LDS (capacity kHash); rows that overflow half of it are
// recorded in `ovf` and left for the GLOBAL = true pass, whose table lives in gk/gv at
// goff[row slot] with capacity goff[s+1] - goff[s].
template <bool GLOBAL>
__global__ __launch_bounds__(kBlock) void k_esc_block(
    const int32_t *rows, int32_t nrows, const int32_t *xrp, const int32_t *xcol,
    const double *xval, const int32_t *xpref, const int32_t *yrp, const int32_t *ycol,
    const double *yval, const int64_t *poff, int32_t *ocol, double *oval, int32_t *ucnt,
    int32_t *ovf, int32_t *novf, int32_t *gk, double *gv, const int64_t *goff) {
  __shared__ uint64_t sk[kChunk];
  __shared__ double sv[kChunk];
  __shared__ int32_t lhk[GLOBAL ? 1 : kHash];
  __shared__ double lhv[GLOBAL ? 1 : kHash];
  __shared__ int32_t s_cnt, s_ovf;
  __shared__ int32_t s_scan[kBlock];
  const int tid = threadIdx.x;
  const int32_t slot = blockIdx.x;
  if (slot >= nrows) return;  // block-uniform
  const int32_t i = rows[slot];
  const int32_t xb = xrp[i], xe = xrp[i + 1];
  const int64_t base = poff[i];
  const int32_t T = (int32_t)(poff[i + 1] - base);
  const bool single = T <= kChunk;
  int32_t *hk;
  double *hv;
  int32_t cap;
  if (GLOBAL) {
    hk = gk + goff[slot];
    hv = gv + goff[slot];
    cap = (int32_t)(goff[slot + 1] - goff[slot]);
  } else {
    hk = lhk;
    hv = lhv;
    cap = kHash;
  }
  if (tid == 0) {
    s_cnt = 0;
    s_ovf = 0;
  }
  if (!single)
    for (int32_t q = tid; q < cap; q += kBlock) hk[q] = -1;
  __syncthreads();

  for (int32_t c0 = 0; c0 < T; c0 += kChunk) {
    const int32_t L = min(kChunk, T - c0);
    const int32_t Lp = next_pow2(L);
    for (int32_t q = tid; q < Lp; q += kBlock) {
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
    if (single) {
      // heads of equal-column runs; each head sums its run in position order
      int32_t nh = 0;
      for (int32_t r = tid * 4; r < tid * 4 + 4; ++r)
        if (r < L && (r == 0 || (sk[r] >> 32) != (sk[r - 1] >> 32))) ++nh;
      s_scan[tid] = nh;
      __syncthreads();
      for (int off = 1; off < kBlock; off <<= 1) {
        const int32_t add = (tid >= off) ? s_scan[tid - off] : 0;
        __syncthreads();
        s_scan[tid] += add;
        __syncthreads();
      }
      int32_t idx = s_scan[tid] - nh;
      for (int32_t r = tid * 4; r < tid * 4 + 4; ++r) {
        if (r < L && (r == 0 || (sk[r] >> 32) != (sk[r - 1] >> 32))) {
          const uint32_t key = (uint32_t)(sk[r] >> 32);
          double sum = 0.0;
          for (int32_t q = r; q < L && (uint32_t)(sk[q] >> 32) == key; ++q)
            sum += sv[(uint32_t)sk[q]];
          ocol[base + idx] = (int32_t)key;
          oval[base + idx] = sum;
          ++idx;
        }
      }
      if (tid == kBlock - 1) ucnt[i] = s_scan[kBlock - 1];
      return;  // single chunk: done (block-uniform)
    }
    // chunked: each distinct column of the chunk is accumulated by its head into the table
    for (int32_t r = tid; r < L; r += kBlock) {
      const uint32_t key = (uint32_t)(sk[r] >> 32);
      if (r > 0 && (uint32_t)(sk[r - 1] >> 32) == key) continue;
      const uint32_t msk = (uint32_t)cap - 1;
      uint32_t h = hash_slot((int32_t)key, msk);
      bool fresh = false;
      for (int32_t probe = 0; probe < cap; ++probe) {
        const int32_t old = atomicCAS(&hk[h], -1, (int32_t)key);
        if (old == -1) {
          fresh = true;
          break;
        }
        if (old == (int32_t)key) break;
        h = (h + 1) & msk;
      }
      double acc = fresh ? 0.0 : hv[h];
      for (int32_t q = r; q < L && (uint32_t)(sk[q] >> 32) == key; ++q)
        acc += sv[(uint32_t)sk[q]];
      hv[h] = acc;
      if (fresh) {
        const int32_t c = atomicAdd(&s_cnt, 1);
        if (2 * (c + 1) > cap) s_ovf = 1;
      }
    }
    __syncthreads();
    if (s_ovf) break;  // block-uniform
  }
  if (s_ovf) {
    if (tid == 0) ovf[atomicAdd(novf, 1)] = i;
    return;
  }
  bitonic_kv(hk, hv, cap);
  const int32_t U = s_cnt;
  for (int32_t r = tid; r < U; r += kBlock) {
    ocol[base + r] = hk[r];
    oval[base + r] = hv[r];
  }
  if (tid == 0) ucnt[i] = U;
}

__global__ void k_ovf_caps(int32_t nov, const int32_t *rows, const int64_t *poff, int32_t ncols,
                           int64_t *caps) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nov) return;
  const int32_t i = rows[s];
  int64_t b = poff[i + 1] - poff[i];
  if (b > ncols) b = ncols;
  int64_t c = 2 * kHash;
  while (c < 2 * b) c <<= 1;
  caps[s] = c;
}

__global__ void k_compact(int32_t m, const int64_t *poff, const int32_t *ucnt,
                          const int32_t *crp, const int32_t *ocol, const double *oval,
                          int32_t *ccol, double *cval) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= m) return;
  const int32_t i = (int32_t)i64;
  const int64_t src = poff[i];
  const int32_t dst = crp[i];
  for (int32_t q = 0; q < ucnt[i]; ++q) {
    ccol[dst + q] = ocol[src + q];
    cval[dst + q] = oval[src + q];
  }
}

void spgemm(const Csr &X, const Csr &Y, Arena &ar, Csr &C, hipStream_t s) {
  const int32_t m = X.n;
  C.n = m;
  C.ncols = Y.ncols;
  Arena tmp;
  tmp.stream = s;
  int64_t *cnt = tmp.alloc<int64_t>(m + 1);
  int32_t *xpref = tmp.alloc<int32_t>(X.nnz > 0 ? X.nnz : 1);
  int64_t *poff = tmp.alloc<int64_t>(m + 1);
  if (m > 0) {
    k_count_products<<<grid_for(m), kBlock, 0, s>>>(m, X.rp, X.col, Y.rp, cnt, xpref);
    SA_LAUNCH_CHECK();
  }
  exclusive_scan_i64(cnt, poff, m, s);
  const int64_t total = read1(poff + m, s);
  int32_t *ocol = tmp.alloc<int32_t>(total > 0 ? total : 1);
  double *oval = tmp.alloc<double>(total > 0 ? total : 1);
  int32_t *ucnt = tmp.alloc<int32_t>(m + 1);
  int32_t *small = tmp.alloc<int32_t>(m > 0 ? m : 1);
  int32_t *big = tmp.alloc<int32_t>(m > 0 ? m : 1);
  int32_t *counters = tmp.alloc<int32_t>(4);
  fill_i32(counters, 0, 4, s);
  if (m > 0) {
    k_bin_rows<<<grid_for(m), kBlock, 0, s>>>(m, poff, small, big, counters);
    SA_LAUNCH_CHECK();
  }
  int32_t hc[4];
  SA_HIP(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
  SA_HIP(hipStreamSynchronize(s));
  const int32_t nsmall = hc[0], nbig = hc[1];
  if (nsmall > 0) {
    k_esc_wave<<<(unsigned)nsmall, kWave, 0, s>>>(small, nsmall, X.rp, X.col, X.val, Y.rp,
                                                   Y.col, Y.val, poff, ocol, oval, ucnt);
    SA_LAUNCH_CHECK();
  }
  if (nbig > 0) {
    int32_t *ovf = tmp.alloc<int32_t>(nbig);
    int32_t *novf = counters + 2;
    k_esc_block<false><<<(unsigned)nbig, kBlock, 0, s>>>(
        big, nbig, X.rp, X.col, X.val, xpref, Y.rp, Y.col, Y.val, poff, ocol, oval, ucnt, ovf,
        novf, nullptr, nullptr, nullptr);
    SA_LAUNCH_CHECK();
    const int32_t nov = read1(novf, s);
    if (nov > 0) {
      int64_t *caps = tmp.alloc<int64_t>(nov + 1);
      int64_t *goff = tmp.alloc<int64_t>(nov + 1);
      k_ovf_caps<<<grid_for(nov), kBlock, 0, s>>>(nov, ovf, poff, Y.ncols, caps);
      SA_LAUNCH_CHECK();
      exclusive_scan_i64(caps, goff, nov, s);
      const int64_t gtot = read1(goff + nov, s);
      int32_t *gk = tmp.alloc<int32_t>(gtot);
      double *gv = tmp.alloc<double>(gtot);
      k_esc_block<true><<<(unsigned)nov, kBlock, 0, s>>>(
          ovf, nov, X.rp, X.col, X.val, xpref, Y.rp, Y.col, Y.val, poff, ocol, oval, ucnt,
          ovf, counters + 3, gk, gv, goff);
      SA_LAUNCH_CHECK();
    }
  }
  C.rp = ar.alloc<int32_t>(m + 1);
  exclusive_scan_i32(ucnt, C.rp, m, s);
  C.nnz = read1(C.rp + m, s);
  C.col = ar.alloc<int32_t>(C.nnz);
  C.val = ar.alloc<double>(C.nnz);
  if (m > 0) {
    k_compact<<<grid_for(m), kBlock, 0, s>>>(m, poff, ucnt, C.rp, ocol, oval, C.col, C.val);
    SA_LAUNCH_CHECK();
  }
}

}  // namespace sa
