// Device-side bodies of the solve-phase kernels (internal).
//
// Every solve kernel exists twice: a standalone launch over one vector or matrix
// (solve_kernels.hip) and a grouped launch over a table of segments, one per hierarchy
// (solve_batch.hip).  Both call the functions below with the segment's own arguments, so a
// hierarchy's arithmetic is the same whichever way its work was launched.
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace sa {

// Epilogues with a block_max member also reduce a per-row value over the row block:
// row_max(has_row, s, pre) is called by every thread, block_max(b, m) once per block.
template <class E, class = void>
struct HasBlockMax : std::false_type {};
template <class E>
struct HasBlockMax<E, std::void_t<decltype(&E::block_max)>> : std::true_type {};

template <class T>
struct Chunk {
  static constexpr int value = sizeof(T) == 8 ? 2048 : 4096;
};

constexpr int32_t kPlanWindow = 2048;  // cost units per SpMV block
constexpr int32_t kPlanRowCost = 8;     // cost of a row besides its entries

// Row sums.  A row of at most kLongRow = 64 entries is summed in ascending column order from
// 0.  A longer row is summed the same way by its own thread when Split is false (the plain
// definition, used where the result must equal the sequential sum bit for bit), and
// otherwise, with in-row positions k = 0..L-1 in ascending column order, as 64 interleaved
// partial sums p_l over the positions l, l+64, l+128, ... (each in order from 0), followed by
// p_0 + ... + p_63 in order from 0.  For L <= 64 the two forms agree exactly; the split lets
// lane l of a wavefront form p_l instead of one thread adding all L products in a dependent
// chain.
constexpr int32_t kLongRow = 64;

// The rows of a row block start within one window of kPlanWindow cost units (row r costs
// rp[r] + kPlanRowCost r, at least its entry count), and a chunk holds kPlanWindow entries:
// every row of a block but its last lies in the block's first chunk, so at most one row (the
// last) spans chunks.
static_assert(Chunk<double>::value >= kPlanWindow && Chunk<float>::value >= kPlanWindow,
              "rows other than a block's last fit its first chunk");

// LDS of one SpMV row block: the chunk's products (a long row that lies in the chunk gets
// its 64 partial sums written over its own first 64 products), the partials of a long row
// that spans chunks, and per wavefront the mask of its threads whose rows are long.
template <class T>
struct SpmvShared {
  T prod[Chunk<T>::value];
  T lastp[64];
  uint64_t longmask[kBlock / 64];
};

// One SpMV row block b (rows plan[2b] .. plan[2b+2]-1, entries from plan[2b+1]): the block
// streams the rows' entries through LDS in coalesced chunks, forming each product
// val*x[col] once.  Every thread adds the products of its own short row in ascending column
// order from 0.  The block's j-th long row is taken by wavefront j mod 4: lane l forms p_l
// (carried in a register across chunks for the one row that spans chunks) and stores it in
// LDS; after the chunk's barrier the row's own thread adds its 64 partials in order.  Each
// row's sum goes to the epilogue from the row's own thread.
template <class T, class Epi, bool Split = true>
__device__ __forceinline__ void spmv_block(int32_t b, const int32_t *__restrict__ plan,
                                           const int32_t *__restrict__ rp,
                                           const int32_t *__restrict__ col,
                                           const T *__restrict__ val,
                                           const T *__restrict__ x, const Epi &epi,
                                           SpmvShared<T> &sh) {
  constexpr int CH = Chunk<T>::value;
  constexpr int NW = kBlock / 64;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  // row and entry ranges: two independent 8-byte loads (one round trip)
  const int2 p0 = ((const int2 *)plan)[b], p1 = ((const int2 *)plan)[b + 1];
  const int32_t r0 = p0.x, e0 = p0.y, r1 = p1.x, e1 = p1.y;
  if (r0 >= r1) {  // block-uniform: no rows (a block max, if any, is 0)
    if constexpr (HasBlockMax<Epi>::value)
      if (t == 0) epi.block_max(b, 0ull);
    return;
  }
  const int32_t row = r0 + t;
  int32_t mb = 0, me = 0;
  typename Epi::Pre pre{};
  if (row < r1) {
    mb = rp[row];
    me = rp[row + 1];
    pre = epi.load(row);  // the epilogue's vector reads overlap the entry loads
  }
  T s = T(0);
  T cp = T(0);       // p_lane of the long row that continues into the next chunk
  bool lng = false;  // this thread's row is long
  bool any = false;  // block-uniform: the block has long rows
  for (int32_t c0 = e0; c0 < e1; c0 += CH) {
    const int32_t c1 = min(c0 + CH, e1);
#pragma unroll 8
    for (int32_t e = c0 + t; e < c1; e += kBlock) sh.prod[e - c0] = val[e] * x[col[e]];
    if (c0 == e0) {
      // classified after the first chunk's loads are issued, so the row-pointer reads
      // overlap them (the empty asm keeps the compiler from hoisting the test, and with it
      // the wait for mb and me, above the loop)
      int32_t b2 = mb, e2 = me;
      asm volatile("" : "+v"(b2), "+v"(e2));
      lng = Split && e2 - b2 > kLongRow;
      const uint64_t lmask = __ballot(lng);
      if (lane == 0) sh.longmask[wv] = lmask;
      any = __syncthreads_or(lng) != 0;
    } else {
      __syncthreads();
    }
    if (!lng) {
      // in-order sum of the row's products in this chunk; loads are issued 8 at a time
      // ahead of the (sequential) adds
      int32_t e = max(mb, c0);
      const int32_t en = min(me, c1);
      for (; e + 8 <= en; e += 8) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = sh.prod[e - c0 + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) s += v[q];
      }
      for (; e < en; ++e) s += sh.prod[e - c0];
    }
    // long rows: this wavefront's share, in row order (block-uniform masks)
    int32_t j = 0;
#pragma unroll 1
    for (int q = 0; q < (any ? NW : 0); ++q) {
      uint64_t m = sh.longmask[q];
      while (m) {
        const int bit = __builtin_ctzll(m);
        m &= m - 1;
        if ((j++ & (NW - 1)) != wv) continue;  // wave-uniform
        const int32_t rb = rp[r0 + q * 64 + bit], re = rp[r0 + q * 64 + bit + 1];
        const int32_t lo = max(rb, c0), hi = min(re, c1);
        if (lo >= hi) continue;  // no entries in this chunk
        // this lane's positions k = lane (mod 64) in [lo, hi), 4 loads ahead of the adds
        const int32_t k0 = lo - rb;
        int32_t e = lo + ((lane - k0) & 63);
        T acc = rb < c0 ? cp : T(0);
        for (; e + 192 < hi; e += 256) {
          const T a0 = sh.prod[e - c0], a1 = sh.prod[e + 64 - c0];
          const T a2 = sh.prod[e + 128 - c0], a3 = sh.prod[e + 192 - c0];
          acc += a0;
          acc += a1;
          acc += a2;
          acc += a3;
        }
        for (; e < hi; e += 64) acc += sh.prod[e - c0];
        if (re > c1) cp = acc;                         // continues into the next chunk
        else if (rb >= c0) sh.prod[rb - c0 + lane] = acc;  // over this lane's first product
        else sh.lastp[lane] = acc;                      // a spanning row ends here
      }
    }
    __syncthreads();
    if (any) {  // block-uniform: long rows ending in this chunk add their partials in order
      if (lng && me > c0 && me <= c1) {
        const T *pj = mb >= c0 ? sh.prod + (mb - c0) : sh.lastp;
#pragma unroll 1
        for (int l = 0; l < 64; l += 8) {
          T v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = pj[l + q];
#pragma unroll
          for (int q = 0; q < 8; ++q) s += v[q];
        }
      }
      if (c1 < e1) __syncthreads();  // before the next chunk's products
    }
  }
  if (row < r1) epi.store(row, s, pre);
  if constexpr (HasBlockMax<Epi>::value) {
    // the block's largest epilogue value: wavefront maxima, then thread 0 over the four (the
    // long-row masks' words are free by now)
    unsigned long long m = epi.row_max(row < r1, s, pre);
    for (int off = 32; off >= 1; off >>= 1) {
      const unsigned long long o = __shfl_xor(m, off, 64);
      m = o > m ? o : m;
    }
    if (lane == 0) sh.longmask[wv] = m;
    __syncthreads();
    if (t == 0) {
      unsigned long long mb2 = sh.longmask[0];
#pragma unroll
      for (int q = 1; q < NW; ++q) mb2 = sh.longmask[q] > mb2 ? sh.longmask[q] : mb2;
      epi.block_max(b, mb2);
    }
  }
}

// ---- fused SpMV epilogues: row i receives s = (A x)_i ------------------------------------
// load(i) reads the row's other inputs (issued before the row's entries are gathered, so
// their latency overlaps); store(i, s, pre) computes and writes.  Inputs are never vectors
// the same launch writes at another row.
template <class T>
struct EpStore {
  T *y;
  struct Pre {};
  __device__ Pre load(int32_t) const { return {}; }
  __device__ void store(int32_t i, T s, const Pre &) const { y[i] = s; }
};
template <class T>
struct EpScale {
  const T *d;
  T *y;
  struct Pre {
    T d;
  };
  __device__ Pre load(int32_t i) const { return {d[i]}; }
  __device__ void store(int32_t i, T s, const Pre &p) const { y[i] = p.d * s; }
};
// y = d (A x) as EpScale, and the largest |y_i| (NaN left out) as the bit pattern of a
// non-negative double (monotone for non-negative values): each row block adds its maximum
// with one atomic maximum to slot (block mod kMaxSlots).
template <class T>
struct EpScaleMax {
  const T *d;
  T *y;
  unsigned long long *slots;
  struct Pre {
    T d;
  };
  __device__ Pre load(int32_t i) const { return {d[i]}; }
  __device__ void store(int32_t i, T s, const Pre &p) const { y[i] = p.d * s; }
  __device__ unsigned long long row_max(bool has, T s, const Pre &p) const {
    if (!has) return 0ull;
    const double a = fabs((double)(p.d * s));
    return (a == a) ? (unsigned long long)__double_as_longlong(a) : 0ull;
  }
  __device__ void block_max(int32_t b, unsigned long long m) const {
    if (m != 0ull) atomicMax(slots + (b % kMaxSlots), m);
  }
};
template <class T>
struct EpResid {
  const T *f;
  T *r;
  struct Pre {
    T f;
  };
  __device__ Pre load(int32_t i) const { return {f[i]}; }
  __device__ void store(int32_t i, T s, const Pre &p) const { r[i] = p.f - s; }
};
template <class T>
struct EpAdd {
  T *u;
  struct Pre {
    T u;
  };
  __device__ Pre load(int32_t i) const { return {u[i]}; }
  __device__ void store(int32_t i, T s, const Pre &p) const { u[i] = p.u + s; }
};
template <class T>
struct EpChebStart {
  const T *f, *invD;
  T theta;
  T *r, *d;
  struct Pre {
    T f, invD;
  };
  __device__ Pre load(int32_t i) const { return {f[i], invD[i]}; }
  __device__ void store(int32_t i, T s, const Pre &p) const {
    T ri = p.f - s;
    r[i] = ri;
    d[i] = (p.invD * ri) / theta;
  }
};
template <class T>
struct EpChebStep {
  const T *d, *rin, *invD;
  T *rout, *u, *dout;
  T c1, c2;
  bool uzero, last;
  struct Pre {
    T d, rin, invD, u;
  };
  __device__ Pre load(int32_t i) const {
    return {d[i], rin[i], invD[i], uzero ? T(0) : u[i]};
  }
  __device__ void store(int32_t i, T s, const Pre &p) const {
    T di = p.d;
    T ui = p.u + di;
    T ri = p.rin - s;
    rout[i] = ri;
    T dn = c1 * di + c2 * (p.invD * ri);
    if (last) {
      u[i] = ui + dn;
    } else {
      u[i] = ui;
      dout[i] = dn;
    }
  }
};
template <class T>
struct EpJacobi {
  const T *u, *f, *invD;
  T w;
  T *u2;
  struct Pre {
    T u, f, invD;
  };
  __device__ Pre load(int32_t i) const { return {u[i], f[i], invD[i]}; }
  __device__ void store(int32_t i, T s, const Pre &p) const {
    T r = p.f - s;
    u2[i] = p.u + w * (p.invD * r);
  }
};

// ---- element-wise bodies -----------------------------------------------------------------
template <class T>
__device__ __forceinline__ void cheb_first_at(int32_t i, const T *f, const T *invD, T theta,
                                              T *d, T *u, bool write_u) {
  T di = (invD[i] * f[i]) / theta;
  d[i] = di;
  if (write_u) u[i] = T(0) + di;
}
template <class T>
__device__ __forceinline__ void vec_add_at(int32_t i, T *u, const T *d) {
  u[i] = u[i] + d[i];
}
template <class T>
__device__ __forceinline__ void jacobi_first_at(int32_t i, const T *f, const T *invD, T w,
                                                T *u) {
  u[i] = T(0) + w * (invD[i] * f[i]);
}
__device__ __forceinline__ void update_xr_at(int32_t i, double *x, double *r, const double *p,
                                             const double *q, double a) {
  x[i] = x[i] + a * p[i];
  r[i] = r[i] - a * q[i];
}
__device__ __forceinline__ void update_p_at(int32_t i, double *p, const double *z, double beta) {
  p[i] = z[i] + beta * p[i];
}
__device__ __forceinline__ void vec_sub_at(int32_t i, const double *z, const double *zo,
                                           double *w) {
  w[i] = z[i] - zo[i];
}

// ---- canonical inner product: one block of 4096 terms --------------------------------------
// Lane t of 256 sums terms t + 256 m (m = 0..15) sequentially from 0 (products x[i]*y[i], or
// x[i] alone when y is null), then s[t] += s[t + w] for w = 128 ... 1.
__device__ __forceinline__ void dot_block(int64_t blk, const double *__restrict__ x,
                                          const double *__restrict__ y, int64_t n,
                                          double *__restrict__ out, double *sh) {
  const int t = threadIdx.x;
  const int64_t base = blk * 4096 + t;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    int64_t i = base + 256 * m;
    if (i < n) acc += (y ? x[i] * y[i] : x[i]);
  }
  sh[t] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (t < w) sh[t] = sh[t] + sh[t + w];
    __syncthreads();
  }
  if (t == 0) *out = sh[0];
}

// ---- dense GEMV row (coarsest level): one wavefront per row --------------------------------
__device__ __forceinline__ void gemv_row(int64_t row, int32_t n, const double *__restrict__ M,
                                         const double *__restrict__ x,
                                         double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const double *m = M + row * n;
  double acc = 0.0;
  for (int32_t j = lane; j < n; j += 64) acc += m[j] * x[j];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[row] = acc;
}

// ---- PCG scalar steps ------------------------------------------------------------------------
__device__ __forceinline__ void pcg_alpha_on(PcgScalars *S) {
  if (!(S->pq > 0.0)) S->err = 1;
  S->alpha = S->rho / S->pq;
}
__device__ __forceinline__ void pcg_beta_on(PcgScalars *S, bool pr) {
  if (!(S->rho1 > 0.0)) S->err = 2;
  S->beta = (pr ? S->rw : S->rho1) / S->rho;
  S->rho = S->rho1;
}
__device__ __forceinline__ void pcg_init_on(PcgScalars *S) {
  if (!(S->rho1 > 0.0)) S->err = 2;
  S->rho = S->rho1;
}

}  // namespace sa
