// CPU oracle for the SA-AMG setup and PCG solve -- TEST INFRASTRUCTURE ONLY.
//
// Plain, single-threaded, obviously-ordered code written from the paper (Hu, Siefert,
// Tuminaro, arXiv 2103.10476).  Only tests, the smoke check and the benchmark's CPU
// baseline load it.  Built with -O2 -ffp-contract=off and no fast-math, so every
// floating-point operation below happens exactly as written.
//
// Readings of the paper where it is silent or ambiguous are marked "Reading:" in the
// comments.  The arithmetic order of every floating-point reduction is fixed here and
// stated in the comments (every row sum, y = A x included, runs sequentially in ascending
// column order starting from 0.0; inner products use the canonical 4096/256 tree of
// canon_sum), because the GPU library reproduces those orders to give bit-identical setups.
//
// Parity status per function: every step is pinned by tests against printed values,
// closed forms, invariants or dense brute force, except the aggregation order reading (a
// reading, pinned by the paper's Fig. 1 examples and by the equivalence of the greedy
// definition with distance-2 maximal independent sets).

#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

enum {
  ST_OK = 0,
  ST_NOT_CONVERGED = 1,
  ST_INVALID = -1,
  ST_BAD_CSR = -2,
  ST_NONPOS_DIAG = -3,
  ST_NEG_EIG = -4,
  ST_STALLED = -5,
  ST_COARSE = -6,
  ST_BREAKDOWN = -9,
};

enum { V_SPRSFY = 1, V_OFFLMP = 2, V_1NORM = 4, V_CNSTRNT = 8 };

// mask codes per stored entry of A
enum : uint8_t { M_WEAK = 0, M_STRONG = 1, M_DROPPED = 2, M_DIAG = 3 };

struct Csr {
  int nr = 0, nc = 0;
  std::vector<int32_t> rp, col;
  std::vector<double> val;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

Csr make_csr(int32_t n, int32_t ncols, const int32_t *rp, const int32_t *col,
             const double *val) {
  Csr a;
  a.nr = n;
  a.nc = ncols;
  a.rp.assign(rp, rp + n + 1);
  a.col.assign(col, col + rp[n]);
  if (val) a.val.assign(val, val + rp[n]);
  return a;
}

// ------------------------------------------------------------------------------------
// Counter-based generator: splitmix64 (Steele, Lea, Flood, OOPSLA 2014), output number k
// of the sequence started at `seed`.
// ------------------------------------------------------------------------------------
uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Stream keys: (stream << 56) | (level << 40) | index.
// Stream 0: start vector of the prolongator eigenvalue estimate; 1: smoother estimate;
// 2: hashed aggregation order.
uint64_t stream_key(int stream, int level, int64_t i) {
  return ((uint64_t)stream << 56) | ((uint64_t)level << 40) | (uint64_t)i;
}

// Canonical reduction tree used for every inner product (a fixed convention, since the
// paper does not fix summation order): blocks of 4096 terms; within a block, lane t of 256
// sums terms t, t+256, ..., t+15*256 sequentially from 0.0; then s[t] += s[t+w] for
// w = 128, 64, ..., 1; the block results are reduced again by the same rule until one
// value remains.
double canon_sum(std::vector<double> cur) {
  do {
    size_t nb = (cur.size() + 4095) / 4096;
    if (nb == 0) nb = 1;
    std::vector<double> next(nb);
    for (size_t b = 0; b < nb; ++b) {
      double s[256];
      for (int t = 0; t < 256; ++t) {
        s[t] = 0.0;
        for (int m = 0; m < 16; ++m) {
          size_t idx = b * 4096 + (size_t)t + 256 * (size_t)m;
          if (idx < cur.size()) s[t] += cur[idx];
        }
      }
      for (int w = 128; w >= 1; w /= 2)
        for (int t = 0; t < w; ++t) s[t] = s[t] + s[t + w];
      next[b] = s[0];
    }
    cur.swap(next);
  } while (cur.size() > 1);
  return cur[0];
}

double dot(const std::vector<double> &x, const std::vector<double> &y) {
  std::vector<double> p(x.size());
  for (size_t i = 0; i < x.size(); ++i) p[i] = x[i] * y[i];
  return canon_sum(p);
}

// y = A x, the plain definition: y_i = sum over the row's stored entries of A_ij x_j, the
// products added sequentially in ascending column order from 0.0 (the paper fixes no order;
// this is the textbook one).
void spmv(const Csr &A, const std::vector<double> &x, std::vector<double> &y) {
  y.assign(A.nr, 0.0);
  for (int i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) s += A.val[e] * x[A.col[e]];
    y[i] = s;
  }
}

int check_csr(int32_t n, const int32_t *rp, const int32_t *col, const double *val) {
  if (n < 0 || !rp) return fail(ST_INVALID, "bad n or rp");
  if (rp[0] != 0) return fail(ST_BAD_CSR, "rp[0] != 0");
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return fail(ST_BAD_CSR, "row pointers decrease");
    bool diag = false;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return fail(ST_BAD_CSR, "column out of range");
      if (e > rp[i] && col[e] <= col[e - 1]) return fail(ST_BAD_CSR, "columns not ascending");
      if (col[e] == i) diag = true;
      if (val && !std::isfinite(val[e])) return fail(ST_INVALID, "non-finite value");
    }
    if (!diag) return fail(ST_BAD_CSR, "missing diagonal");
  }
  return ST_OK;
}

double diag_of(const Csr &A, int i) {
  for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
    if (A.col[e] == i) return A.val[e];
  return 0.0;
}

// ------------------------------------------------------------------------------------
// Strength of connection (Sec. 1.1, strength criterion): off-diagonal (i,j) is strong iff
// |A_ij| >= theta*sqrt(A_ii*A_jj).  Reading: evaluated squared, a*a >= (theta*theta)*
// (A_ii*A_jj), with a non-positive product A_ii*A_jj meaning weak; equal to the printed
// test except at exact ties and independent of a correctly rounded sqrt.
// ------------------------------------------------------------------------------------
void strength(const Csr &A, double theta, std::vector<uint8_t> &mask) {
  std::vector<double> d(A.nr);
  for (int i = 0; i < A.nr; ++i) d[i] = diag_of(A, i);
  double th2 = theta * theta;
  mask.assign(A.nnz(), M_WEAK);
  for (int i = 0; i < A.nr; ++i) {
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      int j = A.col[e];
      if (j == i) {
        mask[e] = M_DIAG;
        continue;
      }
      double a = A.val[e];
      double p = d[i] * d[j];
      bool strong = (p > 0.0) && (a * a >= th2 * p);
      mask[e] = strong ? M_STRONG : M_WEAK;
    }
  }
}

// ------------------------------------------------------------------------------------
// Distance-Laplacian strength (Sec. 3.1): the labels come from a matrix L with A's pattern,
// off-diagonals -w_ij with w_ij the reciprocal of the distance between the coordinates of i
// and j, and the diagonal making each row sum zero; (i,j) is strong iff
// |L_ij| >= theta sqrt(L_ii L_jj).  Readings: the squared distance d2 is summed over the
// coordinates in order from 0.0; w_ij = 1/sqrt(d2) (power 1, the paper's text) or 1/d2
// (power 2, no square root); every stored off-diagonal of A counts, explicit zeros included;
// L_ii = the sum of the row's w_ij in ascending column order from 0.0; the test is evaluated
// squared as for A; coincident coordinates of two connected nodes are an error.
// ------------------------------------------------------------------------------------
int distance_strength(const Csr &A, const std::vector<double> &xyz, int dim, double theta,
                      int power, std::vector<uint8_t> &mask) {
  std::vector<double> w(A.nnz(), 0.0), Ld(A.nr, 0.0);
  for (int i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.col[e];
      if (j == i) continue;
      double d2 = 0.0;
      for (int k = 0; k < dim; ++k) {
        const double t = xyz[(size_t)i * dim + k] - xyz[(size_t)j * dim + k];
        d2 += t * t;
      }
      if (!(d2 > 0.0)) return fail(ST_INVALID, "coincident coordinates of connected nodes");
      w[e] = power == 1 ? 1.0 / std::sqrt(d2) : 1.0 / d2;
      s += w[e];
    }
    Ld[i] = s;
  }
  const double th2 = theta * theta;
  mask.assign(A.nnz(), M_WEAK);
  for (int i = 0; i < A.nr; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.col[e];
      if (j == i) {
        mask[e] = M_DIAG;
        continue;
      }
      const double p = Ld[i] * Ld[j];
      mask[e] = ((p > 0.0) && (w[e] * w[e] >= th2 * p)) ? M_STRONG : M_WEAK;
    }
  return ST_OK;
}

// Coarse coordinates: the centroid of each aggregate's members (Reading: the members'
// coordinates summed in ascending vertex order from 0.0, divided by the member count).
std::vector<double> coarse_coords(const std::vector<double> &xyz, int dim,
                                  const std::vector<int32_t> &agg, int nc) {
  std::vector<double> sum((size_t)nc * dim, 0.0);
  std::vector<int64_t> cnt(nc, 0);
  for (size_t i = 0; i < agg.size(); ++i) {
    if (agg[i] < 0) continue;
    for (int k = 0; k < dim; ++k) sum[(size_t)agg[i] * dim + k] += xyz[i * dim + k];
    ++cnt[agg[i]];
  }
  for (int J = 0; J < nc; ++J)
    for (int k = 0; k < dim; ++k) sum[(size_t)J * dim + k] = sum[(size_t)J * dim + k] / (double)cnt[J];
  return sum;
}

// Aggregation graph G: the strong off-diagonals, symmetrised (G = S u S^T).  Reading: the
// paper treats symmetric matrices; the union keeps the graph undirected when rounding makes
// a coarse matrix's strength pattern slightly unsymmetric.
std::vector<std::vector<int>> strength_graph(const Csr &A, const std::vector<uint8_t> &mask) {
  std::vector<std::vector<int>> g(A.nr);
  for (int i = 0; i < A.nr; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
      if (mask[e] == M_STRONG || mask[e] == M_DROPPED) {
        g[i].push_back(A.col[e]);
        g[A.col[e]].push_back(i);
      }
  for (auto &row : g) {
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
  }
  return g;
}

// ------------------------------------------------------------------------------------
// Aggregation (Sec. 1.1, aggregates; Sec. 2.5 describes the procedure).  Phase 1: visit
// vertices in priority order; a vertex becomes a root when it and all of its strong
// neighbours are unaggregated; the root and its strong neighbours form its aggregate.
// Reading (order): natural index order by default (reproduces Fig. 1's aggregates);
// option: a hashed order, priority (30-bit splitmix64 hash, index).
// Reading (leftovers): every still-unaggregated vertex joins the phase-1 aggregate it has
// the most strong connections to, ties to the smaller aggregate number; phase 1 leaves no
// vertex without an aggregated neighbour, so no new aggregates are needed.
// Reading (isolated vertices, no strong connection at all): by default such a vertex joins
// no aggregate (agg = -1, a zero row of the tentative prolongator) and the smoother alone
// treats it.  This departs from the covering property of Sec. 1.1 (aggregates): with
// `singletons` set, the root rule is applied to it as to any other vertex -- nothing around
// it is aggregated -- so it becomes the root of a singleton aggregate, as the paper's text
// has it.  The covering form carries such vertices unchanged to every coarser level, where
// a whole plane of them (the stretched cubes) stalls the coarsening above the dense coarse
// solver's limit and their zero row sums give zero or negative filtered diagonals.
// Reading (numbering): aggregate number = rank of its root's vertex index among roots.
// ------------------------------------------------------------------------------------
int aggregate(const std::vector<std::vector<int>> &G, int order, uint64_t seed, int level,
              bool singletons, std::vector<int32_t> &agg, std::vector<uint8_t> &is_root) {
  int n = (int)G.size();
  std::vector<int> vis(n);
  for (int v = 0; v < n; ++v) vis[v] = v;
  if (order == 1) {
    std::vector<uint64_t> pri(n);
    for (int v = 0; v < n; ++v)
      pri[v] = ((splitmix64(seed, stream_key(2, level, v)) >> 34) << 32) | (uint64_t)v;
    std::sort(vis.begin(), vis.end(), [&](int a, int b) { return pri[a] < pri[b]; });
  }
  std::vector<int> owner(n, -1);  // root vertex of the phase-1 aggregate, -1 = free
  is_root.assign(n, 0);
  for (int v : vis) {
    if (owner[v] != -1 || (G[v].empty() && !singletons)) continue;
    bool all_free = true;
    for (int u : G[v])
      if (owner[u] != -1) {
        all_free = false;
        break;
      }
    if (!all_free) continue;
    is_root[v] = 1;
    owner[v] = v;
    for (int u : G[v]) owner[u] = v;
  }
  std::vector<int> id(n, -1);
  int nc = 0;
  for (int v = 0; v < n; ++v)
    if (is_root[v]) id[v] = nc++;
  std::vector<int32_t> agg1(n, -1);
  for (int v = 0; v < n; ++v)
    if (owner[v] != -1) agg1[v] = id[owner[v]];
  agg = agg1;
  for (int v = 0; v < n; ++v) {
    if (agg1[v] != -1 || G[v].empty()) continue;
    std::map<int, int> count;
    for (int u : G[v])
      if (agg1[u] != -1) count[agg1[u]] += 1;
    int best = -1, bestc = 0;
    for (auto &kv : count)  // ascending aggregate number: strict > keeps the smallest on ties
      if (kv.second > bestc) {
        best = kv.first;
        bestc = kv.second;
      }
    if (best < 0) return fail(ST_INVALID, "aggregation left a vertex without neighbours");
    agg[v] = best;
  }
  return nc;
}

// ------------------------------------------------------------------------------------
// Sprsfy (Sec. 2.5).  For aggregate J with root r: candidates = aggregates reached by the
// root's weak connections in the graph of A, minus the aggregates reached by its strong
// connections and J itself.  For each candidate c, if exactly one strong connection leads
// from a non-root member of J into c, that entry and its transpose are dropped (relabelled
// weak for the filtered matrix).  Reading: the count is taken over all non-root members of
// J together; decisions use the strength labels from before any drop.
// ------------------------------------------------------------------------------------
void sprsfy(const Csr &A, std::vector<uint8_t> &mask, const std::vector<int32_t> &agg,
            const std::vector<uint8_t> &is_root, int nc) {
  int n = A.nr;
  std::vector<std::vector<int>> members(nc);
  std::vector<int> root(nc, -1);
  for (int v = 0; v < n; ++v) {
    if (agg[v] < 0) continue;
    members[agg[v]].push_back(v);
    if (is_root[v]) root[agg[v]] = v;
  }
  auto is_strong = [&](int32_t e) { return mask[e] == M_STRONG || mask[e] == M_DROPPED; };
  std::vector<std::pair<int, int>> drops;  // (row, entry index)
  for (int J = 0; J < nc; ++J) {
    int r = root[J];
    std::set<int> weak_aggs, strong_aggs;
    strong_aggs.insert(J);
    for (int32_t e = A.rp[r]; e < A.rp[r + 1]; ++e) {
      if (A.col[e] == r) continue;
      if (agg[A.col[e]] < 0) continue;
      if (is_strong(e)) strong_aggs.insert(agg[A.col[e]]);
      else weak_aggs.insert(agg[A.col[e]]);
    }
    std::set<int> cand;
    for (int c : weak_aggs)
      if (!strong_aggs.count(c)) cand.insert(c);
    if (cand.empty()) continue;
    std::map<int, std::vector<std::pair<int, int32_t>>> edges;  // c -> (v, entry)
    for (int v : members[J]) {
      if (v == r) continue;
      for (int32_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
        int u = A.col[e];
        if (u == v || !is_strong(e) || agg[u] < 0) continue;
        if (cand.count(agg[u])) edges[agg[u]].push_back({v, e});
      }
    }
    for (auto &kv : edges) {
      if (kv.second.size() != 1) continue;
      int v = kv.second[0].first;
      int32_t e = kv.second[0].second;
      drops.push_back({v, e});
      int u = A.col[e];
      for (int32_t f = A.rp[u]; f < A.rp[u + 1]; ++f)
        if (A.col[f] == v) drops.push_back({u, f});
    }
  }
  for (auto &d : drops)
    if (mask[d.second] == M_STRONG) mask[d.second] = M_DROPPED;
}

// ------------------------------------------------------------------------------------
// Filtered matrix (Sec. 1.1, filtered matrix; Sec. 2.3, alternative lumping).
// Kept set K_i = strong off-diagonals not dropped; removed set R_i = the other stored
// off-diagonals.  The pattern of the filtered row is {i} u K_i (kept zeros stay stored).
// r_i = sum of the removed entries, ascending from 0.0.
// Plain: diagonal = A_ii + r_i, kept entries copied.
// OffLmp (Algorithm 2, the lumping that avoids small diagonals), with these readings:
//   r_i >= 0  -> as plain (the r_i = 0 case takes this branch, avoiding 0/0);
//   |r_i| <= kappa+ -> kept positives scaled by (1 + r_i/kappa+);
//   otherwise kept positives become 0, rhat = r_i + kappa+, and
//     K- nonempty: r* = largest value in [0, min(|rhat|, A_ii)] with
//        ddom(row) = (c - r*)/(A_ii - r*) <= tau*ddom(A_i), c = -kappa- - rhat; if none,
//        the r* in that interval minimising ddom; diagonal A_ii - r*, kept negatives
//        scaled by 1 + (rhat + r*)/kappa-  (magnitude form of the printed rule; the text's
//        closed form uses the opposite sign convention);
//     K- empty: the whole r_i goes to the kept positives (they turn negative) when that
//        keeps ddom within the bound, else the removed entries are dropped without
//        lumping (row sum not kept);
//   A_ii <= 0 (ddom undefined) -> as plain.
// ddom(A_i) = sum_{j != i} |A_ij| / A_ii over the original row, summed ascending.
// ------------------------------------------------------------------------------------
void lump_row(const Csr &A, int i, const std::vector<uint8_t> &mask, bool offlmp, double tau,
              std::vector<int32_t> &cols, std::vector<double> &vals) {
  cols.clear();
  vals.clear();
  double aii = 0.0;
  int diag_slot = -1;
  double r = 0.0;
  for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
    int j = A.col[e];
    if (j == i) {
      aii = A.val[e];
      diag_slot = (int)cols.size();
      cols.push_back(j);
      vals.push_back(A.val[e]);
    } else if (mask[e] == M_STRONG) {
      cols.push_back(j);
      vals.push_back(A.val[e]);
    } else {
      r += A.val[e];
    }
  }
  if (!offlmp || r >= 0.0 || !(aii > 0.0)) {
    vals[diag_slot] = aii + r;
    return;
  }
  double kp = 0.0, km = 0.0;
  bool has_kp = false, has_km = false;
  for (size_t t = 0; t < cols.size(); ++t) {
    if ((int)t == diag_slot) continue;
    if (vals[t] > 0.0) {
      kp += vals[t];
      has_kp = true;
    } else if (vals[t] < 0.0) {
      km += vals[t];
      has_km = true;
    }
  }
  if (-r <= kp) {
    double delta = r / kp;
    for (size_t t = 0; t < cols.size(); ++t)
      if ((int)t != diag_slot && vals[t] > 0.0) vals[t] = vals[t] * (1.0 + delta);
    return;
  }
  double offsum = 0.0;
  for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
    if (A.col[e] != i) offsum += std::fabs(A.val[e]);
  double T = tau * (offsum / aii);
  double rhat = r + kp;
  if (!has_km) {
    if (has_kp && std::fabs(r + kp) / aii <= T) {
      double delta = r / kp;
      for (size_t t = 0; t < cols.size(); ++t)
        if ((int)t != diag_slot && vals[t] > 0.0) vals[t] = vals[t] * (1.0 + delta);
    }
    return;  // otherwise: removed entries dropped, nothing lumped
  }
  double a = aii;
  double c = -km - rhat;
  double U = std::fmin(std::fabs(rhat), a);
  double bnd = T * a - c;  // feasible r: r*(T-1) <= bnd
  double rs = 0.0;
  bool feasible;
  if (T > 1.0) {
    double ub = bnd / (T - 1.0);
    feasible = ub >= 0.0;
    if (feasible) rs = std::fmin(U, ub);
  } else if (T < 1.0) {
    double lb = bnd / (T - 1.0);
    feasible = lb <= U;
    if (feasible) rs = U;
  } else {
    feasible = bnd >= 0.0;
    if (feasible) rs = U;
  }
  if (!feasible) rs = (c <= a) ? U : 0.0;
  double delta = (rhat + rs) / km;
  for (size_t t = 0; t < cols.size(); ++t) {
    if ((int)t == diag_slot) continue;
    if (vals[t] > 0.0) vals[t] = 0.0;
    else if (vals[t] < 0.0) vals[t] = vals[t] * (1.0 + delta);
  }
  vals[diag_slot] = a - rs;
}

Csr lump(const Csr &A, const std::vector<uint8_t> &mask, bool offlmp, double tau) {
  Csr B;
  B.nr = A.nr;
  B.nc = A.nc;
  B.rp.assign(A.nr + 1, 0);
  std::vector<int32_t> c;
  std::vector<double> v;
  for (int i = 0; i < A.nr; ++i) {
    lump_row(A, i, mask, offlmp, tau, c, v);
    B.col.insert(B.col.end(), c.begin(), c.end());
    B.val.insert(B.val.end(), v.begin(), v.end());
    B.rp[i + 1] = (int32_t)B.col.size();
  }
  return B;
}

// ------------------------------------------------------------------------------------
// Smoothing diagonal.  Plain: the filtered diagonal (Sec. 1.1), zero is an error.
// 1Norm (Sec. 2.1 absolute row sum; Sec. 2.2 safeguard): D = sum_j |Abar_ij| ascending;
// D = 0 -> 1; otherwise with s = sum_j Abar_ij, D := m*s when D < m*s, where
// m = 4/(3(1-sigma)) (= 2 for sigma = 1/3, the value the paper uses), applied to all rows.
// ------------------------------------------------------------------------------------
double safeguard_mult(double sigma) {
  return (sigma == 1.0 / 3.0) ? 2.0 : 4.0 / (3.0 * (1.0 - sigma));
}

int diag(const Csr &Ab, bool one_norm, double sigma, std::vector<double> &invD) {
  invD.assign(Ab.nr, 0.0);
  double m = safeguard_mult(sigma);
  for (int i = 0; i < Ab.nr; ++i) {
    double D;
    if (!one_norm) {
      D = diag_of(Ab, i);
      if (D == 0.0) return fail(ST_NONPOS_DIAG, "zero diagonal in the filtered matrix");
    } else {
      D = 0.0;
      for (int32_t e = Ab.rp[i]; e < Ab.rp[i + 1]; ++e) D += std::fabs(Ab.val[e]);
      if (D == 0.0) {
        D = 1.0;
      } else {
        double s = 0.0;
        for (int32_t e = Ab.rp[i]; e < Ab.rp[i + 1]; ++e) s += Ab.val[e];
        if (D < m * s) D = m * s;
      }
    }
    invD[i] = 1.0 / D;
  }
  return ST_OK;
}

// ------------------------------------------------------------------------------------
// Power method for the largest eigenvalue of invD*M (Sec. 1.1 damping; Sec. 3.1 uses 10
// power sweeps).  Reading: start x_i = 2u-1 with u in [0,1) the top 53 bits of splitmix64;
// each step y = invD .* (M x) (row sums ascending, then the multiply); the estimate is the
// Rayleigh quotient (x.y)/(x.x) of the last step, which can come out negative (the failure
// mode reported in Sec. 3.1); iterates are rescaled by an exact power of two,
// x = y * 2^(-ilogb(max|y_i|)).
// ------------------------------------------------------------------------------------
int power_method(const Csr &M, const std::vector<double> &invD, int iters, uint64_t seed,
                 int level, int stream, double &lambda) {
  int n = M.nr;
  std::vector<double> x(n), y;
  for (int i = 0; i < n; ++i) {
    uint64_t z = splitmix64(seed, stream_key(stream, level, i));
    double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    x[i] = 2.0 * u - 1.0;
  }
  lambda = 0.0;
  for (int t = 1; t <= iters; ++t) {
    spmv(M, x, y);
    for (int i = 0; i < n; ++i) y[i] = invD[i] * y[i];
    if (t == iters) {
      lambda = dot(x, y) / dot(x, x);
      break;
    }
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = std::fmax(mx, std::fabs(y[i]));
    if (!(mx > 0.0) || !std::isfinite(mx)) {
      lambda = 0.0;
      break;
    }
    int e = std::ilogb(mx);
    for (int i = 0; i < n; ++i) x[i] = std::ldexp(y[i], -e);
  }
  if (!(lambda > 0.0) || !std::isfinite(lambda))
    return fail(ST_NEG_EIG, "eigenvalue estimate not positive");
  return ST_OK;
}

// ------------------------------------------------------------------------------------
// Smoothed prolongator (Sec. 1.1, prolongator smoothing): P = (I - omega invD Abar) Ptent
// with Ptent(i, agg_i) = 1 (Sec. 1.1, near null space = constants).  Row i: acc[J] = sum of
// Abar_ik over k in the row with agg_k = J (ascending k, from 0.0); P_iJ = [J == agg_i] -
// (omega*invD_i)*acc[J]; columns = the distinct aggregates reached, ascending.
// ------------------------------------------------------------------------------------
Csr prolongator(const Csr &Ab, const std::vector<double> &invD, const std::vector<int32_t> &agg,
                int nc, double omega) {
  Csr P;
  P.nr = Ab.nr;
  P.nc = nc;
  P.rp.assign(Ab.nr + 1, 0);
  for (int i = 0; i < Ab.nr; ++i) {
    std::map<int, double> acc;
    for (int32_t e = Ab.rp[i]; e < Ab.rp[i + 1]; ++e) {
      int J = agg[Ab.col[e]];
      if (J < 0) continue;  // unaggregated (isolated) vertex: zero tentative row
      auto it = acc.find(J);
      if (it == acc.end()) acc[J] = 0.0 + Ab.val[e];
      else it->second += Ab.val[e];
    }
    double t = omega * invD[i];
    for (auto &kv : acc) {
      double pt = (kv.first == agg[i]) ? 1.0 : 0.0;
      P.col.push_back(kv.first);
      P.val.push_back(pt - t * kv.second);
    }
    P.rp[i + 1] = (int32_t)P.col.size();
  }
  return P;
}

// ------------------------------------------------------------------------------------
// Cnstrnt (Sec. 2.4, Algorithm 3, constraining one prolongator row).  Readings: the loop
// runs while some entry of w is < 0 OR > 1 (the printed AND would never fix a row with only
// negative violators, contradicting the text); argmin/argmax ties go to the lowest column;
// w = nonzero entries, pinned entries leave w but stay stored; rows without violations are
// untouched; infeasible rows (sum < 0 or sum > |w|) and the degenerate w-empty-with-
// residual case take the tentative row (1 at agg_i, 0 elsewhere on the pattern); a zero
// row sum gives the zero row.
// ------------------------------------------------------------------------------------
void cnstrnt_row(const int32_t *cols, double *v, int m, int agg_i) {
  bool viol = false;
  for (int k = 0; k < m; ++k)
    if (v[k] < 0.0 || v[k] > 1.0) viol = true;
  if (!viol) return;
  std::vector<uint8_t> inw(m);
  int cnt = 0;
  double sum = 0.0;
  for (int k = 0; k < m; ++k) {
    inw[k] = v[k] != 0.0;
    if (inw[k]) {
      ++cnt;
      sum += v[k];
    }
  }
  auto tent = [&]() {
    for (int k = 0; k < m; ++k) v[k] = (cols[k] == agg_i) ? 1.0 : 0.0;
  };
  if (sum < 0.0 || sum > (double)cnt) {
    tent();
    return;
  }
  if (sum == 0.0) {
    for (int k = 0; k < m; ++k) v[k] = 0.0;
    return;
  }
  while (cnt > 0) {
    int kmin = -1, kmax = -1;
    for (int k = 0; k < m; ++k) {
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
      if (delta != 0.0) tent();
      return;
    }
    double q = delta / (double)cnt;
    for (int k = 0; k < m; ++k)
      if (inw[k]) v[k] += q;
  }
}

Csr transpose(const Csr &A) {
  Csr T;
  T.nr = A.nc;
  T.nc = A.nr;
  T.rp.assign(A.nc + 1, 0);
  for (int64_t e = 0; e < A.nnz(); ++e) T.rp[A.col[e] + 1]++;
  for (int j = 0; j < A.nc; ++j) T.rp[j + 1] += T.rp[j];
  T.col.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int32_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.nr; ++i)  // rows ascending, so every row of T ascends
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      int32_t p = pos[A.col[e]]++;
      T.col[p] = i;
      T.val[p] = A.val[e];
    }
  return T;
}

// Row i of X*Y by Gustavson's method: for k in X_i ascending, for j in Y_k ascending,
// acc[j] += X_ik*Y_kj (each product rounded, then added; every acc starts at 0.0).  Output
// columns ascending; cancellations stay stored.
void spgemm_row(const Csr &X, const Csr &Y, int i, std::vector<double> &acc,
                std::vector<int32_t> &mark, std::vector<int32_t> &touched) {
  touched.clear();
  for (int32_t e = X.rp[i]; e < X.rp[i + 1]; ++e) {
    int k = X.col[e];
    double a = X.val[e];
    for (int32_t f = Y.rp[k]; f < Y.rp[k + 1]; ++f) {
      int j = Y.col[f];
      if (mark[j] != i) {
        mark[j] = i;
        acc[j] = 0.0;
        touched.push_back(j);
      }
      acc[j] += a * Y.val[f];
    }
  }
  std::sort(touched.begin(), touched.end());
}

Csr spgemm(const Csr &X, const Csr &Y) {
  Csr C;
  C.nr = X.nr;
  C.nc = Y.nc;
  C.rp.assign(X.nr + 1, 0);
  std::vector<double> acc(Y.nc);
  std::vector<int32_t> mark(Y.nc, -1), touched;
  for (int i = 0; i < X.nr; ++i) {
    spgemm_row(X, Y, i, acc, mark, touched);
    for (int j : touched) {
      C.col.push_back(j);
      C.val.push_back(acc[j]);
    }
    C.rp[i + 1] = (int32_t)C.col.size();
  }
  return C;
}

// ------------------------------------------------------------------------------------
// Hierarchy
// ------------------------------------------------------------------------------------
struct Level {
  Csr A;                      // operator of this level
  Csr As;                     // matrix the prolongator is built from (A, or D_B A D_B)
  std::vector<uint8_t> mask;  // per entry of As
  int64_t nnzG = 0;
  std::vector<int32_t> agg;
  std::vector<uint8_t> is_root;
  int nc = 0;
  Csr Abar;
  std::vector<double> invD;
  double lambda = 0.0, omega = 0.0;
  Csr P, R;
  std::vector<double> sm_invD;
  double sm_lambda = 0.0;
  std::vector<double> chol;  // coarsest only: dense Cholesky factor (row-major, lower), or
                             // the LU factors (unit L strictly below, U on and above)
  std::vector<double> xyz;   // node coordinates (n x dim) when the distance strength is used
  // systems SA (block size bs > 1 or a multi-vector nullspace): node-level graph and labels,
  // the QR tentative prolongator, and this level's nullspace (n x k, row-major)
  int bs = 1;
  Csr Gn;
  std::vector<uint8_t> nmask;
  Csr Pt;
  std::vector<double> B;   // this level's nullspace
  std::vector<double> Bc;  // the next level's (R factors of the aggregates' QR)
};

struct Hier {
  orc_options o;
  std::vector<Level> lv;
  bool scaled = false;
  bool valid = true;  // false after a failed re-setup
  int dim = 0;        // > 0: distance-Laplacian strength from coordinates
  int k = 0;          // > 0: systems SA with a k-vector nullspace (QR tentative prolongator)
};

// Dense Cholesky of the coarsest operator, textbook order: L_jj = sqrt(A_jj - sum_k<j L_jk^2),
// L_ij = (A_ij - sum_k<j L_ik L_jk)/L_jj, sums ascending in k (Sec. 3.1: direct solve on
// the coarsest level).
int cholesky(const Csr &A, std::vector<double> &L) {
  int n = A.nr;
  if (n > 8192) return fail(ST_COARSE, "coarsest level too large for the dense solver");
  std::vector<double> D((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) D[(size_t)i * n + A.col[e]] = A.val[e];
  L.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = D[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return fail(ST_COARSE, "coarse Cholesky pivot not positive");
    double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = D[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  return ST_OK;
}

// Dense LU of the coarsest operator without pivoting (for nonsymmetric operators, solved by
// GMRES), Doolittle's order: u_kj = a_kj - sum_{m<k} l_km u_mj, l_ik = (a_ik - sum_{m<k}
// l_im u_mk)/u_kk, sums ascending in m.  A zero or non-finite pivot is an error.
int lu_factor(const Csr &A, std::vector<double> &F) {
  int n = A.nr;
  if (n > 8192) return fail(ST_COARSE, "coarsest level too large for the dense solver");
  std::vector<double> D((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) D[(size_t)i * n + A.col[e]] = A.val[e];
  F.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    for (int j = k; j < n; ++j) {
      double t = D[(size_t)k * n + j];
      for (int m = 0; m < k; ++m) t -= F[(size_t)k * n + m] * F[(size_t)m * n + j];
      F[(size_t)k * n + j] = t;
    }
    const double ukk = F[(size_t)k * n + k];
    if (!(ukk != 0.0) || !std::isfinite(ukk)) return fail(ST_COARSE, "coarse LU pivot zero");
    for (int i = k + 1; i < n; ++i) {
      double t = D[(size_t)i * n + k];
      for (int m = 0; m < k; ++m) t -= F[(size_t)i * n + m] * F[(size_t)m * n + k];
      F[(size_t)i * n + k] = t / ukk;
    }
  }
  return ST_OK;
}

void lu_solve(const std::vector<double> &F, int n, const std::vector<double> &f,
              std::vector<double> &u) {
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double t = f[i];
    for (int k = 0; k < i; ++k) t -= F[(size_t)i * n + k] * y[k];
    y[i] = t;
  }
  u.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < n; ++k) t -= F[(size_t)i * n + k] * u[k];
    u[i] = t / F[(size_t)i * n + i];
  }
}

// The Cholesky factor reads only the lower triangle, so a nonsymmetric coarsest operator
// would be solved as another matrix; such operators must take the LU solver.  Symmetric
// here: max |a_ij - a_ji| <= 1e-10 max |a_ij| (Galerkin products of a symmetric matrix are
// symmetric up to rounding).
bool nearly_symmetric(const Csr &A) {
  const int n = A.nr;
  std::vector<double> D((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) D[(size_t)i * n + A.col[e]] = A.val[e];
  double amax = 0.0, asym = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      amax = std::max(amax, std::fabs(D[(size_t)i * n + j]));
      asym = std::max(asym, std::fabs(D[(size_t)i * n + j] - D[(size_t)j * n + i]));
    }
  return asym <= 1e-10 * amax;
}

void chol_solve(const std::vector<double> &L, int n, const std::vector<double> &f,
                std::vector<double> &u) {
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double t = f[i];
    for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * y[k];
    y[i] = t / L[(size_t)i * n + i];
  }
  u.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * u[k];
    u[i] = t / L[(size_t)i * n + i];
  }
}

int numeric_level(Hier &H, int l);

// ------------------------------------------------------------------------------------
// Systems SA.  The paper treats scalar PDEs and names systems as future work; this follows
// the standard smoothed aggregation for systems (Vanek, Mandel, Brezina) with these
// readings:
//  * dofs are numbered node-major (dof = bs * node + component);
//  * node I is linked to node J when a row of I has an entry in a column of J; the block
//    strength is F_IJ = sum of a_ij^2 over the bs x bs block (rows ascending, then columns
//    ascending), and (I,J) is strong iff F_IJ^2 >= theta^4 F_II F_JJ, i.e. ||A_IJ||_F >=
//    theta sqrt(||A_II||_F ||A_JJ||_F) (the scalar test for bs = 1); with coordinates the
//    distance Laplacian of the node graph decides instead;
//  * a dof entry between different nodes takes its node pair's label, entries inside a node
//    are kept, the diagonal is the diagonal; lumping, the smoothing diagonal and lambda are
//    the scalar definitions applied to dof rows;
//  * aggregates are formed on the node graph; aggregate J's dofs (members ascending,
//    components ascending) take the rows of B, factored B_J = Q_J R_J by Householder
//    reflections; P_t holds Q_J in columns kJ..kJ+k-1 and the coarse nullspace holds R_J;
//  * P = P_t - (omega invD_i) (Abar P_t)_i per row, on the pattern of Abar P_t;
//  * Sprsfy and Cnstrnt (defined for a scalar constant nullspace) are not available.
// ------------------------------------------------------------------------------------
Csr node_graph(const Csr &A, int bs) {
  const int m = A.nr / bs;
  Csr G;
  G.nr = G.nc = m;
  G.rp.assign(m + 1, 0);
  std::vector<int32_t> cols;
  for (int I = 0; I < m; ++I) {
    cols.clear();
    for (int i = I * bs; i < (I + 1) * bs; ++i)
      for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) cols.push_back(A.col[e] / bs);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    G.col.insert(G.col.end(), cols.begin(), cols.end());
    G.rp[I + 1] = (int32_t)G.col.size();
  }
  return G;
}

int32_t slot_of(const Csr &G, int I, int J) {
  const int32_t *b = &G.col[G.rp[I]], *e = b + (G.rp[I + 1] - G.rp[I]);
  const int32_t *p = std::lower_bound(b, e, J);
  return (p != e && *p == J) ? (int32_t)(G.rp[I] + (p - b)) : -1;
}

void block_strength(const Csr &A, int bs, const Csr &G, double theta,
                    std::vector<uint8_t> &nmask) {
  const int m = G.nr;
  std::vector<double> F(G.col.size(), 0.0);
  for (int I = 0; I < m; ++I)
    for (int i = I * bs; i < (I + 1) * bs; ++i)
      for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
        const int32_t q = slot_of(G, I, A.col[e] / bs);
        F[q] = F[q] + A.val[e] * A.val[e];
      }
  std::vector<double> Fd(m);
  for (int I = 0; I < m; ++I) Fd[I] = F[slot_of(G, I, I)];
  const double th4 = (theta * theta) * (theta * theta);
  nmask.assign(G.col.size(), M_WEAK);
  for (int I = 0; I < m; ++I)
    for (int32_t q = G.rp[I]; q < G.rp[I + 1]; ++q) {
      const int J = G.col[q];
      if (J == I) {
        nmask[q] = M_DIAG;
        continue;
      }
      const double p = Fd[I] * Fd[J];
      nmask[q] = ((p > 0.0) && (F[q] * F[q] >= th4 * p)) ? M_STRONG : M_WEAK;
    }
}

void dof_mask(const Csr &A, int bs, const Csr &G, const std::vector<uint8_t> &nmask,
              std::vector<uint8_t> &mask) {
  mask.assign(A.nnz(), M_WEAK);
  for (int i = 0; i < A.nr; ++i)
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.col[e], I = i / bs, J = j / bs;
      mask[e] = (i == j) ? M_DIAG : (I == J) ? M_STRONG : nmask[slot_of(G, I, J)];
    }
}

// Householder QR of the m x k matrix M (row-major), m >= k: R (k x k, upper) and Q (m x k,
// orthonormal columns) with R's diagonal made non-negative.  Each reflection: sigma = sum of
// squares of the column from the diagonal down (ascending), alpha = -sign(a_jj) sqrt(sigma)
// (+sqrt for a_jj <= 0), v = the column with v_j = a_jj - alpha, H = I - 2 v v^T / (v.v);
// products v.a ascending; Q = H_0 ... H_{k-1} applied to the first k unit vectors.
void house_qr(int m, int k, std::vector<double> &M, std::vector<double> &Q,
              std::vector<double> &R) {
  std::vector<double> V((size_t)m * k, 0.0), vv(k, 0.0);
  for (int j = 0; j < k; ++j) {
    double sigma = 0.0;
    for (int i = j; i < m; ++i) sigma = sigma + M[(size_t)i * k + j] * M[(size_t)i * k + j];
    const double nrm = std::sqrt(sigma);
    if (nrm == 0.0) continue;
    const double ajj = M[(size_t)j * k + j];
    const double alpha = ajj > 0.0 ? -nrm : nrm;
    for (int i = j; i < m; ++i) V[(size_t)i * k + j] = M[(size_t)i * k + j];
    V[(size_t)j * k + j] = ajj - alpha;
    double d = 0.0;
    for (int i = j; i < m; ++i) d = d + V[(size_t)i * k + j] * V[(size_t)i * k + j];
    vv[j] = d;
    if (d == 0.0) continue;
    for (int c = j; c < k; ++c) {
      double t = 0.0;
      for (int i = j; i < m; ++i) t = t + V[(size_t)i * k + j] * M[(size_t)i * k + c];
      const double f = (t + t) / d;
      for (int i = j; i < m; ++i) M[(size_t)i * k + c] = M[(size_t)i * k + c] - f * V[(size_t)i * k + j];
    }
  }
  R.assign((size_t)k * k, 0.0);
  for (int r = 0; r < k; ++r)
    for (int c = r; c < k; ++c) R[(size_t)r * k + c] = M[(size_t)r * k + c];
  Q.assign((size_t)m * k, 0.0);
  for (int c = 0; c < k; ++c) Q[(size_t)c * k + c] = 1.0;
  for (int j = k - 1; j >= 0; --j) {
    if (vv[j] == 0.0) continue;
    for (int c = 0; c < k; ++c) {
      double t = 0.0;
      for (int i = j; i < m; ++i) t = t + V[(size_t)i * k + j] * Q[(size_t)i * k + c];
      const double f = (t + t) / vv[j];
      for (int i = j; i < m; ++i) Q[(size_t)i * k + c] = Q[(size_t)i * k + c] - f * V[(size_t)i * k + j];
    }
  }
  for (int r = 0; r < k; ++r)
    if (R[(size_t)r * k + r] < 0.0) {
      for (int c = 0; c < k; ++c) R[(size_t)r * k + c] = -R[(size_t)r * k + c];
      for (int i = 0; i < m; ++i) Q[(size_t)i * k + r] = -Q[(size_t)i * k + r];
    }
}

// P_t and the coarse nullspace of level l from its node aggregates and its nullspace B.
int tentative_qr(Level &L, int k, std::vector<double> &Bc) {
  const int bs = L.bs, n = L.A.nr, nc = L.nc;
  std::vector<std::vector<int>> members(nc);
  for (int I = 0; I < (int)L.agg.size(); ++I)
    if (L.agg[I] >= 0) members[L.agg[I]].push_back(I);
  Csr &P = L.Pt;
  P.nr = n;
  P.nc = nc * k;
  P.rp.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) P.rp[i + 1] = P.rp[i] + (L.agg[i / bs] >= 0 ? k : 0);
  P.col.assign(P.rp[n], 0);
  P.val.assign(P.rp[n], 0.0);
  Bc.assign((size_t)nc * k * k, 0.0);
  std::vector<double> M, Q, R;
  for (int J = 0; J < nc; ++J) {
    const int rows = (int)members[J].size() * bs;
    if (rows < k) return fail(ST_INVALID, "an aggregate has fewer dofs than nullspace vectors");
    M.assign((size_t)rows * k, 0.0);
    for (int q = 0; q < rows; ++q) {
      const int i = members[J][q / bs] * bs + q % bs;
      for (int c = 0; c < k; ++c) M[(size_t)q * k + c] = L.B[(size_t)i * k + c];
    }
    house_qr(rows, k, M, Q, R);
    for (int q = 0; q < rows; ++q) {
      const int i = members[J][q / bs] * bs + q % bs;
      for (int c = 0; c < k; ++c) {
        P.col[P.rp[i] + c] = J * k + c;
        P.val[P.rp[i] + c] = Q[(size_t)q * k + c];
      }
    }
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) Bc[((size_t)J * k + r) * k + c] = R[(size_t)r * k + c];
  }
  return ST_OK;
}

// P = P_t - (omega invD_i) (Abar P_t)_i on the pattern of Abar P_t.
Csr smooth_tentative(const Csr &Ab, const Csr &Pt, const std::vector<double> &invD,
                     double omega) {
  Csr AP = spgemm(Ab, Pt);
  Csr P = AP;
  for (int i = 0; i < AP.nr; ++i) {
    const double t = omega * invD[i];
    for (int32_t e = AP.rp[i]; e < AP.rp[i + 1]; ++e) {
      double pt = 0.0;
      for (int32_t f = Pt.rp[i]; f < Pt.rp[i + 1]; ++f)
        if (Pt.col[f] == AP.col[e]) pt = Pt.val[f];
      P.val[e] = pt - t * AP.val[e];
    }
  }
  return P;
}

int build_level_system(Hier &H, int l) {
  Level &L = H.lv[l];
  const orc_options &o = H.o;
  L.Gn = node_graph(L.As, L.bs);
  if (H.dim > 0) {
    int st = distance_strength(L.Gn, L.xyz, H.dim, o.theta, o.dist_power, L.nmask);
    if (st) return st;
  } else {
    block_strength(L.As, L.bs, L.Gn, o.theta, L.nmask);
  }
  dof_mask(L.As, L.bs, L.Gn, L.nmask, L.mask);
  auto G = strength_graph(L.Gn, L.nmask);
  L.nnzG = 0;
  for (auto &g : G) L.nnzG += (int64_t)g.size();
  int nc = aggregate(G, o.agg_order, o.seed, l, false, L.agg, L.is_root);
  if (nc < 0) return nc;
  L.nc = nc;
  if (nc == 0) return 1;
  if ((int64_t)nc * H.k >= L.A.nr) return fail(ST_STALLED, "coarsening stalled");
  std::vector<double> Bc;
  int st = tentative_qr(L, H.k, Bc);
  if (st) return st;
  st = numeric_level(H, l);
  if (st) return st;
  L.Bc.swap(Bc);
  return ST_OK;
}

int build_level(Hier &H, int l) {
  if (H.k > 0) return build_level_system(H, l);
  Level &L = H.lv[l];
  const orc_options &o = H.o;
  if (H.dim > 0) {
    int st = distance_strength(L.As, L.xyz, H.dim, o.theta, o.dist_power, L.mask);
    if (st) return st;
  } else {
    strength(L.As, o.theta, L.mask);
  }
  auto G = strength_graph(L.As, L.mask);
  L.nnzG = 0;
  for (auto &g : G) L.nnzG += (int64_t)g.size();
  int nc = aggregate(G, o.agg_order, o.seed, l, o.singletons != 0, L.agg, L.is_root);
  if (nc < 0) return nc;
  L.nc = nc;
  if (L.nnzG == 0) return 1;  // no strong connection left: this level becomes the coarsest
  if (nc >= L.A.nr) return fail(ST_STALLED, "coarsening stalled");
  if (o.variants & V_SPRSFY) sprsfy(L.As, L.mask, L.agg, L.is_root, nc);
  return numeric_level(H, l);
}

// Level l from its strength labels (mask, Sprsfy drops included) and aggregates on: filtered
// matrix, smoothing diagonal, eigenvalue estimate, damping, smoothed prolongator, Cnstrnt.
int numeric_level(Hier &H, int l) {
  Level &L = H.lv[l];
  const orc_options &o = H.o;
  const int nc = L.nc;
  L.Abar = lump(L.As, L.mask, (o.variants & V_OFFLMP) != 0, o.tau);
  bool one_norm = (o.variants & V_1NORM) != 0;
  int st = diag(L.Abar, one_norm, o.sigma, L.invD);
  if (st) return st;
  if (one_norm && o.one_norm_power == 0) {
    L.lambda = 1.0;
  } else {
    st = power_method(L.Abar, L.invD, o.power_iters, o.seed, l, 0, L.lambda);
    if (st) return st;
  }
  L.omega = 4.0 / (3.0 * L.lambda);
  if (H.k > 0) {
    L.P = smooth_tentative(L.Abar, L.Pt, L.invD, L.omega);
    return ST_OK;
  }
  L.P = prolongator(L.Abar, L.invD, L.agg, nc, L.omega);
  if (o.variants & V_CNSTRNT)
    for (int i = 0; i < L.P.nr; ++i)
      cnstrnt_row(&L.P.col[L.P.rp[i]], &L.P.val[L.P.rp[i]], L.P.rp[i + 1] - L.P.rp[i],
                  L.agg[i]);
  return ST_OK;
}

// Reading: a general nullspace vector B is handled by the exact symmetric scaling
// Ahat = D_B A D_B (Ahat_ij = (B_i*A_ij)*B_j), building the hierarchy with constant B on
// Ahat and returning P_1 = D_B Phat_1.  Sets level 0's As (A itself when B is null or ones).
int apply_nullspace(Hier &H, const double *B) {
  Level &L0 = H.lv[0];
  const int n = L0.A.nr;
  L0.As = L0.A;
  H.scaled = false;
  if (!B) return ST_OK;
  bool scaled = false;
  for (int i = 0; i < n; ++i) {
    if (!(B[i] != 0.0) || !std::isfinite(B[i]))
      return fail(ST_INVALID, "nullspace entry zero or non-finite");
    if (B[i] != 1.0) scaled = true;
  }
  if (!scaled) return ST_OK;
  Csr &S = L0.As;
  for (int i = 0; i < n; ++i)
    for (int32_t e = S.rp[i]; e < S.rp[i + 1]; ++e) S.val[e] = (B[i] * S.val[e]) * B[S.col[e]];
  H.scaled = true;
  return ST_OK;
}

// P_1 = D_B Phat_1 (scaled case), R_l = P_l^T, A_{l+1} = R_l (A_l P_l) into level l+1.
void galerkin(Hier &H, int l, const double *B) {
  Level &L = H.lv[l];
  if (l == 0 && H.scaled) {
    Csr &P = L.P;
    for (int i = 0; i < P.nr; ++i)
      for (int32_t e = P.rp[i]; e < P.rp[i + 1]; ++e) P.val[e] = B[i] * P.val[e];
  }
  L.R = transpose(L.P);
  Csr AP = spgemm(L.A, L.P);
  Level &Ln = H.lv[l + 1];
  Ln.A = spgemm(L.R, AP);
  Ln.As = Ln.A;
  if (H.dim > 0) Ln.xyz = coarse_coords(L.xyz, H.dim, L.agg, L.nc);
  if (H.k > 0) {
    Ln.bs = H.k;
    Ln.B = L.Bc;
  }
}

// Smoothers on every level but the coarsest (Sec. 3.1: Chebyshev of degree 2 on
// [lambda/10, lambda], lambda from 10 power sweeps on invD*A), and the coarsest factor.
int finish(Hier &H) {
  const orc_options &o = H.o;
  const int nl = (int)H.lv.size();
  for (int l = 0; l + 1 < nl; ++l) {
    Level &L = H.lv[l];
    L.sm_invD.assign(L.A.nr, 0.0);
    for (int i = 0; i < L.A.nr; ++i) {
      double d = diag_of(L.A, i);
      if (!(d > 0.0)) return fail(ST_NONPOS_DIAG, "non-positive diagonal in a level operator");
      L.sm_invD[i] = 1.0 / d;
    }
    int st = power_method(L.A, L.sm_invD, o.power_iters, o.seed, l, 1, L.sm_lambda);
    if (st) return st;
    L.sm_lambda = L.sm_lambda * o.cheb_boost;
  }
  Level &Lc = H.lv[nl - 1];
  if (Lc.A.nr > 8192) return fail(ST_COARSE, "coarsest level too large for the dense solver");
  if (o.coarse_solver == 1) return lu_factor(Lc.A, Lc.chol);
  if (!nearly_symmetric(Lc.A))
    return fail(ST_COARSE, "coarsest operator not symmetric: use the LU coarse solver");
  return cholesky(Lc.A, Lc.chol);
}

}  // namespace

// =====================================================================================
// C interface
// =====================================================================================
extern "C" {

const char *orc_last_error(void) { return g_err.c_str(); }

void orc_default_options(orc_options *o) {
  std::memset(o, 0, sizeof(*o));
  o->theta = 0.02;
  o->variants = 0;
  o->one_norm_power = 0;
  o->tau = 1.1;
  o->sigma = 1.0 / 3.0;
  o->power_iters = 10;
  o->agg_order = 0;
  o->seed = 12345;
  o->max_levels = 10;
  o->max_coarse = 1000;
  o->smoother = 0;
  o->degree = 2;
  o->cheb_ratio = 10.0;
  o->cheb_boost = 1.0;
  o->rtol = 1e-8;
  o->max_iter = 500;
  o->pcg_beta = 0;
  o->dist_power = 1;
  o->coarse_solver = 0;
  o->singletons = 0;
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t k) { return splitmix64(seed, k); }

double orc_dot(int64_t n, const double *x, const double *y) {
  std::vector<double> p((size_t)n);
  for (int64_t i = 0; i < n; ++i) p[i] = x[i] * y[i];
  return canon_sum(p);
}

int orc_setup(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *B, const orc_options *o, void **out) {
  return orc_setup_coords(n, rp, col, val, B, nullptr, 0, o, out);
}

}  // extern "C"

namespace {
int setup_common(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                 const double *B, int32_t bs, const double *Bm, int32_t k,
                 const double *coords, int32_t dim, const orc_options *o, void **out) {
  *out = nullptr;
  int st = check_csr(n, rp, col, val);
  if (st) return st;
  if (k > 0) {
    if (bs < 1 || bs > 16 || n % bs != 0) return fail(ST_INVALID, "block size");
    if (k > 16) return fail(ST_INVALID, "nullspace dimension");
    if (o->variants & (V_SPRSFY | V_CNSTRNT))
      return fail(ST_INVALID, "Sprsfy and Cnstrnt are not defined for systems");
    for (int64_t q = 0; q < (int64_t)n * k; ++q)
      if (!std::isfinite(Bm[q])) return fail(ST_INVALID, "non-finite nullspace entry");
  }
  if (o->theta < 0.0 || o->theta > 1.0 || o->max_levels < 1 || o->degree < 1 ||
      o->power_iters < 1)
    return fail(ST_INVALID, "bad options");
  if (coords && (dim < 1 || dim > 3)) return fail(ST_INVALID, "coordinate dimension");
  if (o->coarse_solver != 0 && o->coarse_solver != 1) return fail(ST_INVALID, "coarse_solver");
  if (o->dist_power != 1 && o->dist_power != 2) return fail(ST_INVALID, "dist_power");
  const int64_t npts = k > 0 ? n / bs : n;  // coordinates are per node
  for (int64_t q = 0; coords && q < npts * dim; ++q)
    if (!std::isfinite(coords[q])) return fail(ST_INVALID, "non-finite coordinate");
  Hier *H = new Hier();
  H->o = *o;
  H->dim = coords ? dim : 0;
  H->k = k;
  H->lv.emplace_back();
  H->lv[0].A = make_csr(n, n, rp, col, val);
  if (coords) H->lv[0].xyz.assign(coords, coords + (size_t)npts * dim);
  if (k > 0) {
    H->lv[0].bs = bs;
    H->lv[0].B.assign(Bm, Bm + (size_t)n * k);
  }
  st = apply_nullspace(*H, B);
  if (st) {
    delete H;
    return st;
  }
  for (int l = 0;; ++l) {
    Level &L = H->lv[l];
    if (L.A.nr <= o->max_coarse || l + 1 >= o->max_levels) break;
    st = build_level(*H, l);
    if (std::getenv("ORACLE_VERBOSE"))
      std::fprintf(stderr, "oracle level %d: n=%d nnz=%lld nc=%d status=%d\n", l, H->lv[l].A.nr,
                   (long long)H->lv[l].A.nnz(), H->lv[l].nc, st);
    if (st < 0) {
      delete H;
      return st;
    }
    if (st == 1) {  // nothing to aggregate: stop here, level l is the coarsest
      Level &Lc = H->lv[l];
      Lc.mask.clear();
      Lc.agg.clear();
      Lc.is_root.clear();
      Lc.nc = 0;
      break;
    }
    H->lv.emplace_back();
    galerkin(*H, l, B);
  }
  st = finish(*H);
  if (st) {
    delete H;
    return st;
  }
  *out = H;
  return ST_OK;
}
}  // namespace

extern "C" {

int orc_setup_coords(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                     const double *B, const double *coords, int32_t dim, const orc_options *o,
                     void **out) {
  return setup_common(n, rp, col, val, B, 1, nullptr, 0, coords, dim, o, out);
}

int orc_setup_system(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                     int32_t bs, const double *B, int32_t k, const double *coords, int32_t dim,
                     const orc_options *o, void **out) {
  if (!B || k < 1) return fail(ST_INVALID, "systems setup needs a nullspace");
  return setup_common(n, rp, col, val, nullptr, bs, B, k, coords, dim, o, out);
}

// Numeric re-setup: new values on the setup's pattern, with every symbolic decision of the
// setup kept (strength labels and Sprsfy drops, aggregates); the numbers are recomputed by
// the setup's own steps.  On failure the hierarchy is left unusable (solves refuse it).
int orc_resetup(void *h, const double *val, const double *B) {
  Hier *H = (Hier *)h;
  if (H->k > 0 && B) return fail(ST_INVALID, "a systems hierarchy keeps its nullspace");
  Level &L0 = H->lv[0];
  const int n = L0.A.nr;
  H->valid = false;
  for (int64_t e = 0; e < L0.A.nnz(); ++e) {
    if (!std::isfinite(val[e])) return fail(ST_INVALID, "non-finite matrix value");
    L0.A.val[e] = val[e];
  }
  (void)n;
  int st = apply_nullspace(*H, B);
  if (st) return st;
  const int nl = (int)H->lv.size();
  for (int l = 0; l + 1 < nl; ++l) {
    st = numeric_level(*H, l);
    if (st) return st;
    galerkin(*H, l, B);
  }
  st = finish(*H);
  if (st) return st;
  H->valid = true;
  return ST_OK;
}

int orc_num_levels(const void *h) { return (int)((const Hier *)h)->lv.size(); }

int orc_level_block(const void *h, int l, int64_t *s) {
  const Hier *H = (const Hier *)h;
  if (l < 0 || l >= (int)H->lv.size()) return fail(ST_INVALID, "bad level");
  const Level &L = H->lv[l];
  s[0] = L.bs;
  s[1] = H->k;
  s[2] = L.Pt.nnz();
  s[3] = L.Gn.nr;
  s[4] = (int64_t)L.Gn.col.size();
  s[5] = (int64_t)L.B.size();
  return ST_OK;
}

int orc_level_sizes(const void *h, int l, int64_t *s) {
  const Hier *H = (const Hier *)h;
  if (l < 0 || l >= (int)H->lv.size()) return fail(ST_INVALID, "bad level");
  const Level &L = H->lv[l];
  s[0] = L.A.nr;
  s[1] = L.A.nnz();
  s[2] = L.nc;
  s[3] = L.Abar.nnz();
  s[4] = L.P.nnz();
  s[5] = L.R.nnz();
  s[6] = L.nnzG;
  s[7] = (l + 1 == (int)H->lv.size()) ? 1 : 0;
  return ST_OK;
}

int orc_level_scalars(const void *h, int l, double *s) {
  const Hier *H = (const Hier *)h;
  if (l < 0 || l >= (int)H->lv.size()) return fail(ST_INVALID, "bad level");
  const Level &L = H->lv[l];
  s[0] = L.lambda;
  s[1] = L.omega;
  s[2] = L.sm_lambda;
  s[3] = 0.0;
  return ST_OK;
}

int orc_export(const void *h, int l, int what, void *buf) {
  const Hier *H = (const Hier *)h;
  if (l < 0 || l >= (int)H->lv.size()) return fail(ST_INVALID, "bad level");
  const Level &L = H->lv[l];
  auto cp = [&](const void *src, size_t bytes) {
    if (bytes) std::memcpy(buf, src, bytes);
    return ST_OK;
  };
  switch (what) {
    case 0: return cp(L.A.rp.data(), L.A.rp.size() * 4);
    case 1: return cp(L.A.col.data(), L.A.col.size() * 4);
    case 2: return cp(L.A.val.data(), L.A.val.size() * 8);
    case 3: return cp(L.mask.data(), L.mask.size());
    case 4: return cp(L.agg.data(), L.agg.size() * 4);
    case 5: return cp(L.is_root.data(), L.is_root.size());
    case 6: return cp(L.Abar.rp.data(), L.Abar.rp.size() * 4);
    case 7: return cp(L.Abar.col.data(), L.Abar.col.size() * 4);
    case 8: return cp(L.Abar.val.data(), L.Abar.val.size() * 8);
    case 9: return cp(L.invD.data(), L.invD.size() * 8);
    case 10: return cp(L.P.rp.data(), L.P.rp.size() * 4);
    case 11: return cp(L.P.col.data(), L.P.col.size() * 4);
    case 12: return cp(L.P.val.data(), L.P.val.size() * 8);
    case 13: return cp(L.R.rp.data(), L.R.rp.size() * 4);
    case 14: return cp(L.R.col.data(), L.R.col.size() * 4);
    case 15: return cp(L.R.val.data(), L.R.val.size() * 8);
    case 16: return cp(L.sm_invD.data(), L.sm_invD.size() * 8);
    case 17: return cp(L.As.val.data(), L.As.val.size() * 8);
    case 18: return cp(L.xyz.data(), L.xyz.size() * 8);
    case 19: return cp(L.Pt.rp.data(), L.Pt.rp.size() * 4);
    case 20: return cp(L.Pt.col.data(), L.Pt.col.size() * 4);
    case 21: return cp(L.Pt.val.data(), L.Pt.val.size() * 8);
    case 22: return cp(L.B.data(), L.B.size() * 8);
    case 23: return cp(L.nmask.data(), L.nmask.size());
    case 24: return cp(L.Gn.rp.data(), L.Gn.rp.size() * 4);
    case 25: return cp(L.Gn.col.data(), L.Gn.col.size() * 4);
    default: return fail(ST_INVALID, "bad export selector");
  }
}

}  // extern "C"

namespace {

// ------------------------------------------------------------------------------------
// Smoothers (Sec. 3.1: degree-2 Chebyshev on [lambda/10, lambda]; Jacobi is an option).
// Chebyshev semi-iteration in invD*A with theta_c = (lam + lam/ratio)/2,
// delta_c = (lam - lam/ratio)/2, sigma1 = theta_c/delta_c:
//   r = f - A u (r = f when u = 0), rho = 1/sigma1, d = (invD.*r)/theta_c;
//   for m = 1..deg: u += d; stop at m = deg; r -= A d; rho' = 1/(2 sigma1 - rho);
//                   d = (rho' rho) d + (2 rho'/delta_c) (invD.*r); rho = rho'.
// Jacobi: deg sweeps u += omega_J invD.*(f - A u), omega_J = 4/(3 lam) (the paper's
// damping rule of Sec. 1.1 applied to the level operator).
// ------------------------------------------------------------------------------------
void smooth(const Hier &H, int l, const std::vector<double> &f, std::vector<double> &u,
            bool u_zero) {
  const Level &L = H.lv[l];
  const orc_options &o = H.o;
  int n = L.A.nr;
  std::vector<double> r(n), Ad;
  if (o.smoother == 1) {
    double w = 4.0 / (3.0 * L.sm_lambda);
    for (int s = 0; s < o.degree; ++s) {
      if (u_zero && s == 0) {
        r = f;
      } else {
        spmv(L.A, u, Ad);
        for (int i = 0; i < n; ++i) r[i] = f[i] - Ad[i];
      }
      for (int i = 0; i < n; ++i) u[i] = u[i] + w * (L.sm_invD[i] * r[i]);
    }
    return;
  }
  double lam = L.sm_lambda;
  double lo = lam / o.cheb_ratio;
  double thc = (lam + lo) * 0.5;
  double dlc = (lam - lo) * 0.5;
  double s1 = thc / dlc;
  double rho = 1.0 / s1;
  if (u_zero) {
    r = f;
  } else {
    spmv(L.A, u, Ad);
    for (int i = 0; i < n; ++i) r[i] = f[i] - Ad[i];
  }
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = (L.sm_invD[i] * r[i]) / thc;
  for (int m = 1; m <= o.degree; ++m) {
    for (int i = 0; i < n; ++i) u[i] = u[i] + d[i];
    if (m == o.degree) break;
    spmv(L.A, d, Ad);
    for (int i = 0; i < n; ++i) r[i] = r[i] - Ad[i];
    double rho1 = 1.0 / (2.0 * s1 - rho);
    double c1 = rho1 * rho;
    double c2 = (2.0 * rho1) / dlc;
    for (int i = 0; i < n; ++i) d[i] = c1 * d[i] + c2 * (L.sm_invD[i] * r[i]);
    rho = rho1;
  }
}

// V-cycle (Algorithm 1), from a zero initial guess on every level:
// u = S(f, 0); r = f - A u; u_c = V(R r); u += P u_c; u = S(f, u); coarsest: u = A^{-1} f.
void vcycle(const Hier &H, int l, const std::vector<double> &f, std::vector<double> &u) {
  const Level &L = H.lv[l];
  int n = L.A.nr;
  if (l + 1 == (int)H.lv.size()) {
    if (H.o.coarse_solver == 1) lu_solve(L.chol, n, f, u);
    else chol_solve(L.chol, n, f, u);
    return;
  }
  u.assign(n, 0.0);
  smooth(H, l, f, u, true);
  std::vector<double> Au, r(n), fc, uc, Pu;
  spmv(L.A, u, Au);
  for (int i = 0; i < n; ++i) r[i] = f[i] - Au[i];
  spmv(L.R, r, fc);
  vcycle(H, l + 1, fc, uc);
  spmv(L.P, uc, Pu);
  for (int i = 0; i < n; ++i) u[i] = u[i] + Pu[i];
  smooth(H, l, f, u, false);
}

}  // namespace

extern "C" {

int orc_vcycle(const void *h, const double *f, double *u) {
  const Hier *H = (const Hier *)h;
  int n = H->lv[0].A.nr;
  std::vector<double> ff(f, f + n), uu;
  vcycle(*H, 0, ff, uu);
  std::memcpy(u, uu.data(), sizeof(double) * n);
  return ST_OK;
}

// Preconditioned CG (Sec. 3.1-3.3 use CG with the multigrid preconditioner).  Readings:
// x0 = 0; the recurrence residual is tested, dot(r,r) <= (rtol*rtol)*dot(b,b); iteration
// count = k at the first pass; beta Fletcher-Reeves (rho'/rho) or flexible Polak-Ribiere
// (dot(r, z - z_old)/rho).
int orc_solve(const void *h, const double *b, double *x, int32_t *iters, double *relres,
              double *hist) {
  const Hier *H = (const Hier *)h;
  if (!H->valid) return fail(ST_INVALID, "hierarchy left unusable by a failed re-setup");
  const orc_options &o = H->o;
  const Csr &A = H->lv[0].A;
  int n = A.nr;
  std::vector<double> xv(n, 0.0), r(b, b + n), z, p, q, zold;
  double g0 = dot(r, r);
  *iters = 0;
  if (hist) hist[0] = g0;
  if (g0 == 0.0) {
    std::memcpy(x, xv.data(), sizeof(double) * n);
    *relres = 0.0;
    return ST_OK;
  }
  double thr = (o.rtol * o.rtol) * g0;
  vcycle(*H, 0, r, z);
  p = z;
  double rho = dot(r, z);
  if (!(rho > 0.0)) return fail(ST_BREAKDOWN, "preconditioned residual product not positive");
  double rr = g0;
  int status = ST_NOT_CONVERGED;
  int k;
  for (k = 1; k <= o.max_iter; ++k) {
    spmv(A, p, q);
    double pq = dot(p, q);
    if (!(pq > 0.0)) return fail(ST_BREAKDOWN, "p'Ap not positive");
    double alpha = rho / pq;
    for (int i = 0; i < n; ++i) xv[i] = xv[i] + alpha * p[i];
    for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    rr = dot(r, r);
    if (hist) hist[k] = rr;
    if (rr <= thr) {
      status = ST_OK;
      break;
    }
    if (o.pcg_beta == 1) zold = z;
    vcycle(*H, 0, r, z);
    double rho1 = dot(r, z);
    if (!(rho1 > 0.0)) return fail(ST_BREAKDOWN, "preconditioned residual product not positive");
    double beta;
    if (o.pcg_beta == 1) {
      std::vector<double> w(n);
      for (int i = 0; i < n; ++i) w[i] = z[i] - zold[i];
      beta = dot(r, w) / rho;
    } else {
      beta = rho1 / rho;
    }
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rho = rho1;
  }
  *iters = (status == ST_OK) ? k : o.max_iter;
  *relres = std::sqrt(rr / g0);
  std::memcpy(x, xv.data(), sizeof(double) * n);
  return status;
}

// Restarted GMRES(m) with the V-cycle as a right preconditioner, in the flexible form that
// keeps the preconditioned vectors Z (so the update is x += Z y).  The paper solves its
// nonsymmetric wind-turbine pressure systems with GMRES preconditioned by the SA hierarchy
// (Sec. 3.4); it does not fix the GMRES variant, so this follows Saad's textbook algorithm:
//  * x0 = 0, r = b, stop when the least-squares residual |g_{j+1}| <= rtol ||b||;
//  * Arnoldi with classical Gram-Schmidt applied twice (h = V^T w, w -= V h, again, h += h'),
//    each inner product the canonical dot, each element of w -= V h updated with the terms in
//    ascending basis order;
//  * Givens rotations c = a/rho, s = b/rho, rho = sqrt(a*a + b*b) (c = 1, s = 0 when b = 0);
//  * at a restart the true residual b - A x is formed and tested;
//  * a zero new basis norm (lucky breakdown) ends the cycle with the exact Krylov solution.
// Iterations count Arnoldi steps (one V-cycle and one product with A each).
int orc_solve_gmres(const void *h, const double *b, double *x, int32_t restart, int32_t *iters,
                    double *relres, double *hist) {
  const Hier *H = (const Hier *)h;
  if (!H->valid) return fail(ST_INVALID, "hierarchy left unusable by a failed re-setup");
  if (restart < 1) return fail(ST_INVALID, "restart must be positive");
  const orc_options &o = H->o;
  const Csr &A = H->lv[0].A;
  const int n = A.nr;
  const int m = restart;
  std::vector<double> xv(n, 0.0), r(b, b + n);
  const double bn = std::sqrt(dot(r, r));
  *iters = 0;
  if (hist) hist[0] = bn;
  if (bn == 0.0) {
    std::memcpy(x, xv.data(), sizeof(double) * n);
    *relres = 0.0;
    return ST_OK;
  }
  const double target = o.rtol * bn;
  std::vector<std::vector<double>> V(m + 1), Z(m);
  std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), w, c(m + 1);
  auto Hij = [&](int i, int j) -> double & { return Hm[(size_t)i * m + j]; };
  double beta = bn, res = bn;
  int total = 0;
  bool converged = false;
  while (true) {
    V[0].resize(n);
    for (int k = 0; k < n; ++k) V[0][k] = r[k] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    std::fill(Hm.begin(), Hm.end(), 0.0);
    g[0] = beta;
    int kdim = 0;
    for (int j = 0; j < m && total < o.max_iter; ++j) {
      vcycle(*H, 0, V[j], Z[j]);
      spmv(A, Z[j], w);
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= j; ++i) c[i] = dot(V[i], w);
        for (int k = 0; k < n; ++k) {
          double t = w[k];
          for (int i = 0; i <= j; ++i) t = t - c[i] * V[i][k];
          w[k] = t;
        }
        for (int i = 0; i <= j; ++i) Hij(i, j) = pass == 0 ? c[i] : Hij(i, j) + c[i];
      }
      const double hn = std::sqrt(dot(w, w));
      Hij(j + 1, j) = hn;
      if (hn > 0.0) {
        V[j + 1].resize(n);
        for (int k = 0; k < n; ++k) V[j + 1][k] = w[k] / hn;
      }
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
        Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
        Hij(i, j) = t;
      }
      const double a = Hij(j, j), bb = Hij(j + 1, j);
      if (bb == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        const double rho = std::sqrt(a * a + bb * bb);
        cs[j] = a / rho;
        sn[j] = bb / rho;
      }
      Hij(j, j) = cs[j] * a + sn[j] * bb;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      kdim = j + 1;
      res = std::fabs(g[j + 1]);
      if (hist) hist[total] = res;
      if (!std::isfinite(res)) return fail(ST_BREAKDOWN, "GMRES residual not finite");
      if (res <= target || hn == 0.0) {
        converged = true;
        break;
      }
    }
    if (kdim == 0) break;
    // y = H^{-1} g (upper triangular, back substitution with ascending inner sums)
    for (int i = kdim - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < kdim; ++k) t = t - Hij(i, k) * y[k];
      if (Hij(i, i) == 0.0) return fail(ST_BREAKDOWN, "singular GMRES least-squares system");
      y[i] = t / Hij(i, i);
    }
    for (int e = 0; e < n; ++e) {
      double t = xv[e];
      for (int i = 0; i < kdim; ++i) t = t + y[i] * Z[i][e];
      xv[e] = t;
    }
    if (converged || total >= o.max_iter) break;
    spmv(A, xv, w);
    for (int k = 0; k < n; ++k) r[k] = b[k] - w[k];
    beta = std::sqrt(dot(r, r));
    res = beta;
    if (beta <= target) {
      converged = true;
      break;
    }
  }
  *iters = total;
  *relres = res / bn;
  std::memcpy(x, xv.data(), sizeof(double) * n);
  return converged ? ST_OK : ST_NOT_CONVERGED;
}

void orc_destroy(void *h) { delete (Hier *)h; }

// ---- single steps ----------------------------------------------------------------------

int orc_distance_strength(int32_t n, const int32_t *rp, const int32_t *col,
                          const double *coords, int32_t dim, double theta, int32_t dist_power,
                          uint8_t *mask) {
  if (dist_power != 1 && dist_power != 2) return fail(ST_INVALID, "dist_power");
  Csr A = make_csr(n, n, rp, col, nullptr);
  std::vector<double> xyz(coords, coords + (size_t)n * dim);
  std::vector<uint8_t> m;
  int st = distance_strength(A, xyz, dim, theta, dist_power, m);
  if (st) return st;
  std::copy(m.begin(), m.end(), mask);
  return ST_OK;
}

int orc_strength(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                 double theta, uint8_t *mask) {
  int st = check_csr(n, rp, col, val);
  if (st) return st;
  Csr A = make_csr(n, n, rp, col, val);
  std::vector<uint8_t> m;
  strength(A, theta, m);
  std::memcpy(mask, m.data(), m.size());
  return ST_OK;
}

int orc_aggregate(int32_t n, const int32_t *rp, const int32_t *col, const uint8_t *mask,
                  int32_t order, uint64_t seed, int32_t level, int32_t singletons,
                  int32_t *agg, uint8_t *is_root, int32_t *nc) {
  Csr A = make_csr(n, n, rp, col, nullptr);
  std::vector<uint8_t> m(mask, mask + rp[n]);
  auto G = strength_graph(A, m);
  std::vector<int32_t> a;
  std::vector<uint8_t> r;
  int c = aggregate(G, order, seed, level, singletons != 0, a, r);
  if (c < 0) return c;
  std::memcpy(agg, a.data(), sizeof(int32_t) * n);
  std::memcpy(is_root, r.data(), n);
  *nc = c;
  return ST_OK;
}

int orc_sprsfy(int32_t n, const int32_t *rp, const int32_t *col, uint8_t *mask,
               const int32_t *agg, const uint8_t *is_root, int32_t nc) {
  Csr A = make_csr(n, n, rp, col, nullptr);
  std::vector<uint8_t> m(mask, mask + rp[n]);
  std::vector<int32_t> a(agg, agg + n);
  std::vector<uint8_t> r(is_root, is_root + n);
  sprsfy(A, m, a, r, nc);
  std::memcpy(mask, m.data(), m.size());
  return ST_OK;
}

int orc_lump(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
             const uint8_t *mask, int32_t offlmp, double tau, int32_t *out_rp, int32_t *out_col,
             double *out_val) {
  Csr A = make_csr(n, n, rp, col, val);
  std::vector<uint8_t> m(mask, mask + rp[n]);
  Csr B = lump(A, m, offlmp != 0, tau);
  std::memcpy(out_rp, B.rp.data(), sizeof(int32_t) * (n + 1));
  std::memcpy(out_col, B.col.data(), sizeof(int32_t) * B.col.size());
  std::memcpy(out_val, B.val.data(), sizeof(double) * B.val.size());
  return ST_OK;
}

int orc_diag(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
             int32_t one_norm, double sigma, double *invD) {
  Csr A = make_csr(n, n, rp, col, val);
  std::vector<double> d;
  int st = diag(A, one_norm != 0, sigma, d);
  if (st) return st;
  std::memcpy(invD, d.data(), sizeof(double) * n);
  return ST_OK;
}

int orc_spmv(int32_t nr, int32_t nc, const int32_t *rp, const int32_t *col, const double *val,
             const double *x, double *y) {
  Csr A = make_csr(nr, nc, rp, col, val);
  std::vector<double> xv(x, x + nc), yv;
  spmv(A, xv, yv);
  std::memcpy(y, yv.data(), sizeof(double) * nr);
  return ST_OK;
}

int orc_power(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *invD, int32_t iters, uint64_t seed, int32_t level, int32_t stream,
              double *lambda) {
  Csr A = make_csr(n, n, rp, col, val);
  std::vector<double> d(invD, invD + n);
  return power_method(A, d, iters, seed, level, stream, *lambda);
}

int orc_prolongator(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                    const double *invD, const int32_t *agg, double omega, int32_t *out_rp,
                    int32_t *out_col, double *out_val) {
  Csr A = make_csr(n, n, rp, col, val);
  std::vector<double> d(invD, invD + n);
  std::vector<int32_t> a(agg, agg + n);
  int nc = 0;
  for (int i = 0; i < n; ++i) nc = std::max(nc, a[i] + 1);
  Csr P = prolongator(A, d, a, nc, omega);
  std::memcpy(out_rp, P.rp.data(), sizeof(int32_t) * (n + 1));
  std::memcpy(out_col, P.col.data(), sizeof(int32_t) * P.col.size());
  std::memcpy(out_val, P.val.data(), sizeof(double) * P.val.size());
  return ST_OK;
}

int orc_cnstrnt(int32_t n, const int32_t *rp, const int32_t *col, double *val,
                const int32_t *agg) {
  for (int i = 0; i < n; ++i) cnstrnt_row(col + rp[i], val + rp[i], rp[i + 1] - rp[i], agg[i]);
  return ST_OK;
}

int orc_spgemm_row(const int32_t *xrp, const int32_t *xcol, const double *xval,
                   const int32_t *yrp, const int32_t *ycol, const double *yval,
                   int32_t ncols_y, int32_t row, int32_t *out_col, double *out_val) {
  // Works on the row's entries directly (the matrices may be large; nothing is copied).
  std::map<int32_t, double> acc;
  for (int32_t e = xrp[row]; e < xrp[row + 1]; ++e) {
    int k = xcol[e];
    double a = xval[e];
    for (int32_t f = yrp[k]; f < yrp[k + 1]; ++f) {
      int j = ycol[f];
      if (j < 0 || j >= ncols_y) return fail(ST_BAD_CSR, "column out of range");
      auto it = acc.find(j);
      if (it == acc.end()) acc[j] = 0.0 + a * yval[f];
      else it->second += a * yval[f];
    }
  }
  int c = 0;
  for (auto &kv : acc) {
    out_col[c] = kv.first;
    out_val[c] = kv.second;
    ++c;
  }
  return c;
}

}  // extern "C"
