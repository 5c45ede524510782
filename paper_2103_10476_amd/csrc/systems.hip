// Systems SA with a multi-vector nullspace (internal): node graph, block strength, dof labels,
// the QR tentative prolongator and its smoothing.
//
// The paper treats scalar PDEs and names systems as future work; this is the standard
// smoothed aggregation for systems (Vanek, Mandel, Brezina) with these readings:
//  * dofs are numbered node-major (dof = bs * node + component);
//  * node I is linked to node J when a row of I has an entry in a column of J; the block
//    strength is F_IJ = sum of a_ij^2 over the bs x bs block (rows ascending, then columns
//    ascending) and (I,J) is strong iff F_IJ^2 >= theta^4 F_II F_JJ, i.e. ||A_IJ||_F >=
//    theta sqrt(||A_II||_F ||A_JJ||_F) (the scalar test for bs = 1);
//  * a dof entry between two nodes takes the node pair's label; entries inside a node are kept;
//  * aggregate J's dofs (members ascending, components ascending) take the rows of the
//    nullspace B, factored B_J = Q_J R_J by Householder reflections (R's diagonal made
//    non-negative); P_t holds Q_J in columns kJ..kJ+k-1 and the coarse nullspace holds R_J;
//  * P = P_t - (omega invD_i) (Abar P_t)_i per row, on the pattern of Abar P_t.
// Every sum runs in the order stated, so the results equal the sequential definitions bit for
// bit.
#include <climits>

#include "kernels.hpp"

namespace sa {

#define SA_ROW_BEGIN(n)                                              \
  const int64_t i64_ = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; \
  if (i64_ >= (n)) return;                                           \
  const int32_t I = (int32_t)i64_;

constexpr int kMaxBs = 16;

// ---- node graph ------------------------------------------------------------------------------
// Each of node I's bs rows lists its columns ascending, so col / bs is non-decreasing along a
// row: a merge of the bs lists with duplicates removed gives I's neighbours in ascending order.
template <bool FILL>
__global__ void k_node_graph(int32_t m, int32_t bs, const int32_t *rp, const int32_t *col,
                             int32_t *cnt, const int32_t *grp, int32_t *gcol) {
  SA_ROW_BEGIN(m)
  int32_t cur[kMaxBs], end[kMaxBs];
  for (int r = 0; r < bs; ++r) {
    cur[r] = rp[(int64_t)I * bs + r];
    end[r] = rp[(int64_t)I * bs + r + 1];
  }
  int32_t c = 0;
  const int32_t w = FILL ? grp[I] : 0;
  for (;;) {
    int32_t J = INT_MAX;
    for (int r = 0; r < bs; ++r)
      if (cur[r] < end[r]) J = min(J, col[cur[r]] / bs);
    if (J == INT_MAX) break;
    for (int r = 0; r < bs; ++r)
      while (cur[r] < end[r] && col[cur[r]] / bs == J) ++cur[r];
    if (FILL) gcol[w + c] = J;
    ++c;
  }
  if (!FILL) cnt[I] = c;
}

void node_graph(const Csr &A, int32_t bs, Arena &ar, Csr &G, hipStream_t s) {
  if (bs < 1 || bs > kMaxBs) throw Error(SA_ERR_INVALID_ARG, "block size not in 1..16");
  const int32_t m = A.n / bs;
  int32_t *cnt = (int32_t *)dev_alloc(sizeof(int32_t) * (m + 1), s);
  G.n = G.ncols = m;
  G.rp = ar.alloc<int32_t>(m + 1);
  if (m > 0) {
    k_node_graph<false><<<grid_for(m), kBlock, 0, s>>>(m, bs, A.rp, A.col, cnt, nullptr, nullptr);
    SA_LAUNCH_CHECK();
  }
  exclusive_scan_i32(cnt, G.rp, m, s);
  dev_free(cnt, s);
  G.nnz = read1(G.rp + m, s);
  G.col = ar.alloc<int32_t>(G.nnz > 0 ? G.nnz : 1);
  G.val = nullptr;
  if (m > 0) {
    k_node_graph<true><<<grid_for(m), kBlock, 0, s>>>(m, bs, A.rp, A.col, nullptr, G.rp, G.col);
    SA_LAUNCH_CHECK();
  }
}

// ---- block strength ----------------------------------------------------------------------------
__global__ void k_block_F(int32_t m, int32_t bs, const int32_t *rp, const int32_t *col,
                          const double *val, const int32_t *grp, const int32_t *gcol, double *F,
                          double *Fd) {
  SA_ROW_BEGIN(m)
  const int32_t g0 = grp[I], g1 = grp[I + 1];
  for (int32_t q = g0; q < g1; ++q) F[q] = 0.0;
  for (int r = 0; r < bs; ++r) {
    const int64_t i = (int64_t)I * bs + r;
    int32_t q = g0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t J = col[e] / bs;
      while (gcol[q] < J) ++q;  // J is in I's list, which ascends
      F[q] = F[q] + val[e] * val[e];
    }
  }
  double d = 0.0;
  for (int32_t q = g0; q < g1; ++q)
    if (gcol[q] == I) d = F[q];
  Fd[I] = d;
}
__global__ void k_block_label(int32_t m, const int32_t *grp, const int32_t *gcol,
                              const double *F, const double *Fd, double th4, uint8_t *nmask,
                              int32_t *scount) {
  SA_ROW_BEGIN(m)
  int32_t cnt = 0;
  for (int32_t q = grp[I]; q < grp[I + 1]; ++q) {
    const int32_t J = gcol[q];
    if (J == I) {
      nmask[q] = 3;
      continue;
    }
    const double p = Fd[I] * Fd[J];
    const bool strong = (p > 0.0) && (F[q] * F[q] >= th4 * p);
    nmask[q] = strong ? 1 : 0;
    cnt += strong;
  }
  scount[I] = cnt;
}

void block_strength(const Csr &A, int32_t bs, const Csr &G, double theta, uint8_t *nmask,
                    int32_t *scount, hipStream_t s) {
  const int32_t m = G.n;
  if (m <= 0) return;
  Arena tmp;
  tmp.stream = s;
  double *F = tmp.alloc<double>(G.nnz > 0 ? G.nnz : 1);
  double *Fd = tmp.alloc<double>(m);
  k_block_F<<<grid_for(m), kBlock, 0, s>>>(m, bs, A.rp, A.col, A.val, G.rp, G.col, F, Fd);
  const double th4 = (theta * theta) * (theta * theta);
  k_block_label<<<grid_for(m), kBlock, 0, s>>>(m, G.rp, G.col, F, Fd, th4, nmask, scount);
  SA_LAUNCH_CHECK();
}

// ---- dof labels from node labels -----------------------------------------------------------------
__global__ void k_dof_mask(int32_t n, int32_t bs, const int32_t *rp, const int32_t *col,
                           const int32_t *grp, const int32_t *gcol, const uint8_t *nmask,
                           uint8_t *mask) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= n) return;
  const int32_t i = (int32_t)i64, I = i / bs;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
    const int32_t j = col[e], J = j / bs;
    uint8_t lab;
    if (i == j) {
      lab = 3;
    } else if (I == J) {
      lab = 1;
    } else {
      int32_t lo = grp[I], hi = grp[I + 1] - 1;
      lab = 0;
      while (lo <= hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t c = gcol[mid];
        if (c == J) {
          lab = nmask[mid];
          break;
        }
        if (c < J) lo = mid + 1;
        else hi = mid - 1;
      }
    }
    mask[e] = lab;
  }
}
void dof_mask(const Csr &A, int32_t bs, const Csr &G, const uint8_t *nmask, uint8_t *mask,
              hipStream_t s) {
  if (A.n <= 0) return;
  k_dof_mask<<<grid_for(A.n), kBlock, 0, s>>>(A.n, bs, A.rp, A.col, G.rp, G.col, nmask, mask);
  SA_LAUNCH_CHECK();
}

// ---- QR tentative prolongator ----------------------------------------------------------------------
__global__ void k_pt_count(int32_t n, int32_t bs, int32_t k, const int32_t *agg, int32_t *cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = agg[i / bs] >= 0 ? k : 0;
}

// One thread per aggregate; M, V and Q live in the aggregate's slice of the scratch arrays
// (rows x k each, row-major).  err |= ebit when the aggregate has fewer dofs than k.
__global__ void k_agg_qr(int32_t nc, int32_t bs, int32_t k, const int32_t *mrp,
                         const int32_t *mem, const double *B, const int32_t *ptrp,
                         int32_t *ptcol, double *ptval, double *Bc, double *Ms, double *Vs,
                         double *Qs, int32_t *err, int32_t ebit) {
  SA_ROW_BEGIN(nc)
  const int32_t J = I;
  const int32_t m0 = mrp[J], cntn = mrp[J + 1] - m0;
  const int32_t rows = cntn * bs;
  if (rows < k) {
    atomicOr(err, ebit);
    return;
  }
  const int64_t base = (int64_t)m0 * bs * k;
  double *M = Ms + base, *V = Vs + base, *Q = Qs + base;
  auto dof = [&](int32_t q) -> int64_t { return (int64_t)mem[m0 + q / bs] * bs + q % bs; };
  for (int32_t q = 0; q < rows; ++q)
    for (int c = 0; c < k; ++c) {
      M[(int64_t)q * k + c] = B[dof(q) * k + c];
      V[(int64_t)q * k + c] = 0.0;
    }
  double vv[kMaxBs];
  for (int j = 0; j < k; ++j) {
    vv[j] = 0.0;
    double sigma = 0.0;
    for (int32_t i = j; i < rows; ++i) sigma = sigma + M[(int64_t)i * k + j] * M[(int64_t)i * k + j];
    const double nrm = sqrt(sigma);
    if (nrm == 0.0) continue;
    const double ajj = M[(int64_t)j * k + j];
    const double alpha = ajj > 0.0 ? -nrm : nrm;
    for (int32_t i = j; i < rows; ++i) V[(int64_t)i * k + j] = M[(int64_t)i * k + j];
    V[(int64_t)j * k + j] = ajj - alpha;
    double d = 0.0;
    for (int32_t i = j; i < rows; ++i) d = d + V[(int64_t)i * k + j] * V[(int64_t)i * k + j];
    vv[j] = d;
    if (d == 0.0) continue;
    for (int c = j; c < k; ++c) {
      double t = 0.0;
      for (int32_t i = j; i < rows; ++i) t = t + V[(int64_t)i * k + j] * M[(int64_t)i * k + c];
      const double f = (t + t) / d;
      for (int32_t i = j; i < rows; ++i)
        M[(int64_t)i * k + c] = M[(int64_t)i * k + c] - f * V[(int64_t)i * k + j];
    }
  }
  for (int32_t q = 0; q < rows; ++q)
    for (int c = 0; c < k; ++c) Q[(int64_t)q * k + c] = (q == c) ? 1.0 : 0.0;
  for (int j = k - 1; j >= 0; --j) {
    if (vv[j] == 0.0) continue;
    for (int c = 0; c < k; ++c) {
      double t = 0.0;
      for (int32_t i = j; i < rows; ++i) t = t + V[(int64_t)i * k + j] * Q[(int64_t)i * k + c];
      const double f = (t + t) / vv[j];
      for (int32_t i = j; i < rows; ++i)
        Q[(int64_t)i * k + c] = Q[(int64_t)i * k + c] - f * V[(int64_t)i * k + j];
    }
  }
  for (int r = 0; r < k; ++r) {
    const bool flip = M[(int64_t)r * k + r] < 0.0;
    for (int c = 0; c < k; ++c) {
      double rv = (c >= r) ? M[(int64_t)r * k + c] : 0.0;
      if (flip) rv = -rv;
      Bc[((int64_t)J * k + r) * k + c] = rv;
    }
    if (flip)
      for (int32_t q = 0; q < rows; ++q) Q[(int64_t)q * k + r] = -Q[(int64_t)q * k + r];
  }
  for (int32_t q = 0; q < rows; ++q) {
    const int64_t i = dof(q);
    for (int c = 0; c < k; ++c) {
      ptcol[ptrp[i] + c] = J * k + c;
      ptval[ptrp[i] + c] = Q[(int64_t)q * k + c];
    }
  }
}

// The same QR with one wavefront per aggregate and M, V, Q in LDS (rows x k each, rows <=
// maxrows): every sum keeps k_agg_qr's order (one lane runs it from i = j upward), so the
// results are bitwise the same.  Lane 0 forms each Householder vector; the column loops,
// independent across columns, run one lane per column.
__global__ __launch_bounds__(64) void k_agg_qr_lds(int32_t nc, int32_t bs, int32_t k,
                                                   int32_t maxrows, const int32_t *mrp,
                                                   const int32_t *mem, const double *B,
                                                   const int32_t *ptrp, int32_t *ptcol,
                                                   double *ptval, double *Bc, int32_t *err,
                                                   int32_t ebit) {
  extern __shared__ double qr_lds[];
  __shared__ double s_vv[kMaxBs];
  __shared__ int s_skip;
  const int32_t J = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t m0 = mrp[J], cntn = mrp[J + 1] - m0;
  const int32_t rows = cntn * bs;
  if (rows < k) {  // block-uniform
    if (lane == 0) atomicOr(err, ebit);
    return;
  }
  double *M = qr_lds, *V = qr_lds + (int64_t)maxrows * k, *Q = V + (int64_t)maxrows * k;
  auto dof = [&](int32_t q) -> int64_t { return (int64_t)mem[m0 + q / bs] * bs + q % bs; };
  for (int32_t e = lane; e < rows * k; e += 64) {
    const int32_t q = e / k, c = e % k;
    M[e] = B[dof(q) * k + c];
    V[e] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (lane == 0) {
      double vvj = 0.0;
      int skip = 1;
      double sigma = 0.0;
      for (int32_t i = j; i < rows; ++i) sigma = sigma + M[(int64_t)i * k + j] * M[(int64_t)i * k + j];
      const double nrm = sqrt(sigma);
      if (nrm != 0.0) {
        const double ajj = M[(int64_t)j * k + j];
        const double alpha = ajj > 0.0 ? -nrm : nrm;
        for (int32_t i = j; i < rows; ++i) V[(int64_t)i * k + j] = M[(int64_t)i * k + j];
        V[(int64_t)j * k + j] = ajj - alpha;
        double d = 0.0;
        for (int32_t i = j; i < rows; ++i) d = d + V[(int64_t)i * k + j] * V[(int64_t)i * k + j];
        vvj = d;
        skip = d == 0.0;
      }
      s_vv[j] = vvj;
      s_skip = skip;
    }
    __syncthreads();
    if (!s_skip) {
      const int c = j + lane;
      if (c < k) {
        const double d = s_vv[j];
        double t = 0.0;
        for (int32_t i = j; i < rows; ++i) t = t + V[(int64_t)i * k + j] * M[(int64_t)i * k + c];
        const double f = (t + t) / d;
        for (int32_t i = j; i < rows; ++i)
          M[(int64_t)i * k + c] = M[(int64_t)i * k + c] - f * V[(int64_t)i * k + j];
      }
    }
    __syncthreads();
  }
  for (int32_t e = lane; e < rows * k; e += 64) Q[e] = (e / k == e % k) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double vj = s_vv[j];
    if (vj == 0.0) continue;  // block-uniform
    const int c = lane;
    if (c < k) {
      double t = 0.0;
      for (int32_t i = j; i < rows; ++i) t = t + V[(int64_t)i * k + j] * Q[(int64_t)i * k + c];
      const double f = (t + t) / vj;
      for (int32_t i = j; i < rows; ++i)
        Q[(int64_t)i * k + c] = Q[(int64_t)i * k + c] - f * V[(int64_t)i * k + j];
    }
    __syncthreads();
  }
  if (lane < k) {  // row r = lane of R, and the sign of Q's column r
    const int r = lane;
    const bool flip = M[(int64_t)r * k + r] < 0.0;
    for (int c = 0; c < k; ++c) {
      double rv = (c >= r) ? M[(int64_t)r * k + c] : 0.0;
      if (flip) rv = -rv;
      Bc[((int64_t)J * k + r) * k + c] = rv;
    }
    if (flip)
      for (int32_t q = 0; q < rows; ++q) Q[(int64_t)q * k + r] = -Q[(int64_t)q * k + r];
  }
  __syncthreads();
  for (int32_t e = lane; e < rows * k; e += 64) {
    const int32_t q = e / k, c = e % k;
    const int64_t i = dof(q);
    ptcol[ptrp[i] + c] = J * k + c;
    ptval[ptrp[i] + c] = Q[e];
  }
}

void tentative_qr(int32_t n, int32_t bs, int32_t k, const int32_t *agg, int32_t nc,
                  const double *B, Arena &ar, Csr &Pt, double *Bc, int32_t *err, int32_t ebit,
                  hipStream_t s) {
  if (k < 1 || k > kMaxBs) throw Error(SA_ERR_INVALID_ARG, "nullspace dimension not in 1..16");
  const int32_t m = n / bs;
  Arena tmp;
  tmp.stream = s;
  int32_t *cnt = tmp.alloc<int32_t>(n + 1);
  k_pt_count<<<grid_for(n), kBlock, 0, s>>>(n, bs, k, agg, cnt);
  SA_LAUNCH_CHECK();
  Pt.n = n;
  Pt.ncols = nc * k;
  Pt.rp = ar.alloc<int32_t>(n + 1);
  exclusive_scan_i32(cnt, Pt.rp, n, s);
  Pt.nnz = read1(Pt.rp + n, s);
  Pt.col = ar.alloc<int32_t>(Pt.nnz > 0 ? Pt.nnz : 1);
  Pt.val = ar.alloc<double>(Pt.nnz > 0 ? Pt.nnz : 1);
  if (nc <= 0) return;
  int32_t *mrp, *mem;
  member_lists(m, agg, nc, true, tmp, &mrp, &mem, s);
  // one wavefront per aggregate with M, V, Q in LDS when the largest aggregate fits 64 KB
  const int64_t maxrows = (int64_t)max_row_length(nc, mrp, s) * bs;
  const int64_t lds = 3 * maxrows * k * (int64_t)sizeof(double);
  if (lds <= (48 << 10)) {
    k_agg_qr_lds<<<(unsigned)nc, 64, (size_t)lds, s>>>(nc, bs, k, (int32_t)maxrows, mrp, mem, B,
                                                        Pt.rp, Pt.col, Pt.val, Bc, err, ebit);
    SA_LAUNCH_CHECK();
    return;
  }
  const int64_t sz = (int64_t)n * k;
  double *Ms = tmp.alloc<double>(sz), *Vs = tmp.alloc<double>(sz), *Qs = tmp.alloc<double>(sz);
  k_agg_qr<<<grid_for(nc), kBlock, 0, s>>>(nc, bs, k, mrp, mem, B, Pt.rp, Pt.col, Pt.val, Bc, Ms,
                                           Vs, Qs, err, ebit);
  SA_LAUNCH_CHECK();
}

// ---- smoothing: P = P_t - (omega invD_i) (Abar P_t)_i --------------------------------------------
__global__ void k_smooth_pt(int32_t n, const int32_t *aprp, const int32_t *apcol, double *apval,
                            const int32_t *ptrp, const int32_t *ptcol, const double *ptval,
                            const double *invD, const double *omega) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i64 >= n) return;
  const int32_t i = (int32_t)i64;
  const double t = (*omega) * invD[i];
  for (int32_t e = aprp[i]; e < aprp[i + 1]; ++e) {
    double pt = 0.0;
    for (int32_t f = ptrp[i]; f < ptrp[i + 1]; ++f)
      if (ptcol[f] == apcol[e]) pt = ptval[f];
    apval[e] = pt - t * apval[e];
  }
}
void smooth_tentative(const Csr &abar, const Csr &Pt, const double *invD, const double *omega,
                      Arena &ar, Csr &P, hipStream_t s) {
  spgemm(abar, Pt, ar, P, s);
  if (P.n > 0) {
    k_smooth_pt<<<grid_for(P.n), kBlock, 0, s>>>(P.n, P.rp, P.col, P.val, Pt.rp, Pt.col, Pt.val,
                                                 invD, omega);
    SA_LAUNCH_CHECK();
  }
}

}  // namespace sa
