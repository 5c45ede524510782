// Host runtime and C ABI: hierarchy setup (Sec. 1.1 with the adaptations of Sec. 2), the
// V-cycle of Algorithm 1 with Chebyshev/Jacobi smoothing (Sec. 3.1), and preconditioned CG.
//
// Control crosses to the host only at size readbacks (aggregate count, nnz of each new
// matrix), the root-selection termination flags, error checks, and once per CG iteration
// for the stopping test.  Level data never leaves the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include <map>
#include <mutex>

#include "hierarchy.hpp"

namespace sa {

thread_local std::string g_last_error;

enum ErrBits {
  E_STRUCT = 1,
  E_NODIAG = 2,
  E_NONFINITE = 4,
  E_ZERO_FDIAG = 8,
  E_LAMBDA = 16,
  E_DIAG = 32,
  E_CHOL = 64,
  E_COORD = 128,
  E_ASYM = 256,
  E_QR = 512,
  E_PLAN = 1024,
  E_SPAN = 2048
};

constexpr int32_t kMaxRestart = 1024;  // GMRES restart length limit

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

static int32_t read_err(sa_hierarchy *h) { return read1(h->err, h->stream); }

static void check_err(sa_hierarchy *h, int32_t mask_bits, sa_status code, const char *what) {
  const int32_t e = read_err(h);
  if (e & mask_bits) throw Error(code, what);
}

// Side stream of a main stream, one per (device, main stream) and kept for the process (the
// allocator caches blocks per stream).  The smoother set-up of a finished level runs there
// while the main stream builds the next levels; default priority, non-blocking.
static hipStream_t side_stream(hipStream_t main) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, hipStream_t> streams;
  int dev = 0;
  SA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find({dev, main});
  if (it != streams.end()) return it->second;
  hipStream_t s2 = nullptr;
  SA_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
  streams[{dev, main}] = s2;
  return s2;
}

// `waiter` runs its later work after everything already queued on `first`.
static void stream_after(hipStream_t waiter, hipStream_t first) {
  hipEvent_t ev;
  SA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  SA_HIP(hipEventRecord(ev, first));
  SA_HIP(hipStreamWaitEvent(waiter, ev, 0));
  SA_HIP(hipEventDestroy(ev));
}

static double safeguard_mult(double sigma) {
  return (sigma == 1.0 / 3.0) ? 2.0 : 4.0 / (3.0 * (1.0 - sigma));
}

static void validate_options(const sa_options &o) {
  if (o.struct_size != sizeof(sa_options)) throw Error(SA_ERR_INVALID_ARG, "bad struct_size");
  if (!(o.theta >= 0.0 && o.theta <= 1.0)) throw Error(SA_ERR_INVALID_ARG, "theta not in [0,1]");
  if (o.max_levels < 1 || o.max_levels > 16) throw Error(SA_ERR_INVALID_ARG, "max_levels");
  if (o.degree < 1 || o.degree > 16) throw Error(SA_ERR_INVALID_ARG, "degree");
  if (o.power_iters < 1) throw Error(SA_ERR_INVALID_ARG, "power_iters");
  if (!(o.cheb_ratio > 1.0)) throw Error(SA_ERR_INVALID_ARG, "cheb_ratio must exceed 1");
  if (!(o.rtol > 0.0) || o.max_iter < 0) throw Error(SA_ERR_INVALID_ARG, "rtol/max_iter");
  if (o.precision != SA_FP64 && o.precision != SA_FP32_VCYCLE)
    throw Error(SA_ERR_INVALID_ARG, "precision");
  if (o.variants & ~15u) throw Error(SA_ERR_INVALID_ARG, "unknown variant bits");
  if (o.dist_power != 1 && o.dist_power != 2) throw Error(SA_ERR_INVALID_ARG, "dist_power");
  if (o.coarse_solver != SA_COARSE_CHOLESKY && o.coarse_solver != SA_COARSE_LU)
    throw Error(SA_ERR_INVALID_ARG, "coarse_solver");
  if (o.isolated != SA_ISOLATED_LEFT_OUT && o.isolated != SA_ISOLATED_SINGLETON)
    throw Error(SA_ERR_INVALID_ARG, "isolated");
}

static void copy_in(void *dst, const void *src, size_t bytes, sa_location loc, hipStream_t s) {
  if (!bytes) return;
  SA_HIP(hipMemcpyAsync(dst, src, bytes,
                        loc == SA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}

static void chebyshev_scalars(Level &L, const sa_options &o) {
  const double lam = L.sm_lam;
  const double lo = lam / o.cheb_ratio;
  const double thc = (lam + lo) * 0.5;
  const double dlc = (lam - lo) * 0.5;
  const double s1 = thc / dlc;
  double rho = 1.0 / s1;
  L.cheb_theta = thc;
  L.cheb_c1.clear();
  L.cheb_c2.clear();
  for (int m = 1; m < o.degree; ++m) {
    const double rho1 = 1.0 / (2.0 * s1 - rho);
    L.cheb_c1.push_back(rho1 * rho);
    L.cheb_c2.push_back((2.0 * rho1) / dlc);
    rho = rho1;
  }
  L.jac_w = 4.0 / (3.0 * lam);
}

static Csr copy_csr(const Csr &a, Arena &ar, hipStream_t s) {
  Csr c = a;
  c.rp = ar.alloc<int32_t>(a.n + 1);
  c.col = ar.alloc<int32_t>(a.nnz);
  c.val = ar.alloc<double>(a.nnz);
  SA_HIP(hipMemcpyAsync(c.rp, a.rp, sizeof(int32_t) * (a.n + 1), hipMemcpyDeviceToDevice, s));
  SA_HIP(hipMemcpyAsync(c.col, a.col, sizeof(int32_t) * a.nnz, hipMemcpyDeviceToDevice, s));
  SA_HIP(hipMemcpyAsync(c.val, a.val, sizeof(double) * a.nnz, hipMemcpyDeviceToDevice, s));
  return c;
}

// Copies the values of a freshly computed matrix into an existing one of the same pattern.
static void take_values(const Csr &src, Csr &dst, hipStream_t s) {
  if (src.nnz != dst.nnz || src.n != dst.n)
    throw Error(SA_ERR_INVALID_ARG, "re-setup produced a different sparsity pattern");
  if (src.nnz > 0)
    SA_HIP(hipMemcpyAsync(dst.val, src.val, sizeof(double) * src.nnz, hipMemcpyDeviceToDevice,
                          s));
}

// The numeric part of level l, from the strength labels and aggregates on: filtered matrix
// (plain or OffLmp lumping) and smoothing diagonal, eigenvalue estimate and damping,
// prolongator smoothing and Cnstrnt.  fresh: allocate the level's arrays (setup); otherwise
// overwrite the values of the existing ones, whose patterns do not change (re-setup).
// Numeric part of level l, in three steps (the second can run on the side stream):
// lumping into Abar and the smoothing diagonal; the damping factor from the power method on
// D^-1 Abar; the prolongator.
static void numeric_lump(sa_hierarchy *h, int l, bool fresh) {
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  Level &L = h->lv[l];
  Arena &ar = h->ar;
  const int32_t n = L.A.n;
  Arena tmp;
  tmp.stream = s;
  const bool one_norm = (o.variants & SA_1NORM) != 0;
  if (fresh) {
    L.invD = ar.alloc<double>(n);
    L.lam_d = ar.alloc<double>(2);
    L.omega_d = L.lam_d + 1;
  }
  Csr abar;
  lump(n, L.As.nnz, L.As.rp, L.As.col, L.As.val, L.mask, (o.variants & SA_OFFLMP) != 0, o.tau,
       one_norm, safeguard_mult(o.sigma), L.wave_rows, fresh ? ar : tmp, abar, L.invD, h->err,
       s);
  if (fresh) {
    L.Abar = abar;
    spmv_plan(L.Abar, ar, s);
  } else {
    take_values(abar, L.Abar, s);
  }
}
static void numeric_damping(sa_hierarchy *h, int l, hipStream_t s, int32_t *err) {
  const sa_options &o = h->opt;
  Level &L = h->lv[l];
  const bool unit = (o.variants & SA_1NORM) != 0 && o.one_norm_power == 0;
  if (!unit) power_method(L.Abar, L.invD, o.power_iters, o.seed, l, 0, L.lam_d, s);
  damping(L.lam_d, L.omega_d, unit, err, s);
}
static void numeric_prolong(sa_hierarchy *h, int l, bool fresh) {
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  Level &L = h->lv[l];
  Arena &ar = h->ar;
  Arena tmp;
  tmp.stream = s;
  if (h->k > 0) {  // systems: P = P_t - omega D^-1 Abar P_t
    if (fresh) {
      smooth_tentative(L.Abar, L.Pt, L.invD, L.omega_d, ar, L.P, s);
      spmv_plan(L.P, ar, s);
    } else {
      Csr P;
      smooth_tentative(L.Abar, L.Pt, L.invD, L.omega_d, tmp, P, s);
      take_values(P, L.P, s);
    }
    return;
  }
  if (fresh) {
    prolongator(L.Abar, L.invD, L.agg, L.nc, L.omega_d, ar, L.P, s, L.wave_rows);
  } else {
    Csr P;
    prolongator(L.Abar, L.invD, L.agg, L.nc, L.omega_d, tmp, P, s, L.wave_rows);
    take_values(P, L.P, s);
  }
  if (o.variants & SA_CNSTRNT) cnstrnt(L.P, L.agg, s);
  if (fresh) spmv_plan(L.P, ar, s);
}
static void numeric_level(sa_hierarchy *h, int l, bool fresh) {
  numeric_lump(h, l, fresh);
  check_err(h, E_ZERO_FDIAG, SA_ERR_NONPOSITIVE_DIAG, "zero diagonal in the filtered matrix");
  numeric_damping(h, l, h->stream, h->err);
  check_err(h, E_LAMBDA, SA_ERR_NEGATIVE_EIGENVALUE, "eigenvalue estimate not positive");
  numeric_prolong(h, l, fresh);
}

// Builds level l's strength labels and aggregates, then its numeric part.  Returns false when
// the level has no strong connection left (it becomes the coarsest).
// Systems SA (k-vector nullspace): labels on the node graph (block norms or the distance
// Laplacian of node coordinates), dof labels from them, aggregates of nodes, the QR tentative
// prolongator and the coarse nullspace, then the numeric part.
static bool build_level_system(sa_hierarchy *h, int l) {
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  Level &L = h->lv[l];
  Arena &ar = h->ar;
  const int32_t n = L.A.n, bs = L.bs, m = n / bs;
  Arena tmp;
  tmp.stream = s;
  node_graph(L.As, bs, ar, L.Gn, s);
  L.nmask = ar.alloc<uint8_t>(L.Gn.nnz > 0 ? L.Gn.nnz : 1);
  int32_t *scount = tmp.alloc<int32_t>(m + 1);
  const bool gwave = max_row_length(m, L.Gn.rp, s) > 64 || L.Gn.nnz > 24 * (int64_t)m;
  if (h->dim > 0) {
    double *w = tmp.alloc<double>(L.Gn.nnz > 0 ? L.Gn.nnz : 1);
    double *Ld = tmp.alloc<double>(m);
    distance_weights(m, L.Gn.rp, L.Gn.col, L.xyz, h->dim, o.dist_power, w, Ld, h->err, E_COORD,
                     s);
    check_err(h, E_COORD, SA_ERR_INVALID_ARG, "coincident coordinates of connected nodes");
    strength(m, L.Gn.rp, L.Gn.col, w, Ld, o.theta * o.theta, L.nmask, scount, gwave, s);
  } else {
    block_strength(L.As, bs, L.Gn, o.theta, L.nmask, scount, s);
  }
  L.As.maxrow = L.A.maxrow = max_row_length(n, L.As.rp, s);  // A and As share the pattern
  L.wave_rows = L.As.maxrow > 64 || L.As.nnz > 24 * (int64_t)n;
  L.mask = ar.alloc<uint8_t>(L.As.nnz);
  dof_mask(L.As, bs, L.Gn, L.nmask, L.mask, s);
  int32_t *grp = nullptr, *gcol = nullptr;
  const int64_t nnzG = strength_graph(m, L.Gn.rp, L.Gn.col, L.nmask, scount, gwave, tmp, &grp,
                                      &gcol, s);
  L.agg = ar.alloc<int32_t>(m);
  L.is_root = ar.alloc<uint8_t>(m);
  int32_t *root_vertex = nullptr;
  L.nc = aggregate(m, nnzG, grp, gcol, o.agg_order, o.seed, l, false, L.agg, L.is_root, tmp,
                   &root_vertex, &L.mis_rounds, s);
  if (L.nc == 0) return false;
  if ((int64_t)L.nc * h->k >= n) throw Error(SA_ERR_COARSEN_STALLED, "coarsening stalled");
  L.Bc = ar.alloc<double>((int64_t)L.nc * h->k * h->k);
  tentative_qr(n, bs, h->k, L.agg, L.nc, L.B, ar, L.Pt, L.Bc, h->err, E_QR, s);
  check_err(h, E_QR, SA_ERR_INVALID_ARG, "an aggregate has fewer dofs than nullspace vectors");
  numeric_level(h, l, true);
  return true;
}

static bool build_level(sa_hierarchy *h, int l) {
  if (h->k > 0) return build_level_system(h, l);
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  Level &L = h->lv[l];
  Arena &ar = h->ar;
  const int32_t n = L.A.n;
  Arena tmp;
  tmp.stream = s;
  double *dval = tmp.alloc<double>(n);
  const double *sval = L.As.val;  // the matrix the strength test reads: A, or L^(d)
  if (h->dim > 0) {
    double *w = tmp.alloc<double>(L.As.nnz);
    distance_weights(n, L.As.rp, L.As.col, L.xyz, h->dim, o.dist_power, w, dval, h->err,
                     E_COORD, s);
    check_err(h, E_COORD, SA_ERR_INVALID_ARG, "coincident coordinates of connected nodes");
    sval = w;
  } else {
    find_diag(n, L.As.rp, L.As.col, L.As.val, dval, s);
  }
  // rows long enough to leave thread-per-row kernels serial: one wavefront per row instead
  L.As.maxrow = L.A.maxrow = max_row_length(n, L.As.rp, s);  // A and As share the pattern
  L.wave_rows = L.As.maxrow > 64 || L.As.nnz > 24 * (int64_t)n;
  L.mask = ar.alloc<uint8_t>(L.As.nnz);
  int32_t *scount = tmp.alloc<int32_t>(n + 1);
  strength(n, L.As.rp, L.As.col, sval, dval, o.theta * o.theta, L.mask, scount, L.wave_rows,
           s);
  int32_t *grp = nullptr, *gcol = nullptr;
  const int64_t nnzG = strength_graph(n, L.As.rp, L.As.col, L.mask, scount, L.wave_rows, tmp,
                                      &grp, &gcol, s);
  L.agg = ar.alloc<int32_t>(n);
  L.is_root = ar.alloc<uint8_t>(n);
  int32_t *root_vertex = nullptr;
  if (o.variants & SA_SPRSFY) {  // the drops change the labels lumping reads: in sequence
    L.nc = aggregate(n, nnzG, grp, gcol, o.agg_order, o.seed, l,
                     o.isolated == SA_ISOLATED_SINGLETON, L.agg, L.is_root, tmp, &root_vertex,
                     &L.mis_rounds, s);
    if (nnzG == 0) return false;  // no strong connection: the coarsest level
    if (L.nc >= n) throw Error(SA_ERR_COARSEN_STALLED, "coarsening stalled");
    sprsfy(n, L.As.rp, L.As.col, L.mask, L.agg, root_vertex, L.nc, s);
    numeric_level(h, l, true);
    return true;
  }
  // Lumping needs the labels only, so it runs before the aggregation, and the power method
  // for the damping factor runs on the side stream (its own error word) while the root
  // selection runs here.  Errors are checked in the sequential order afterwards; a level that
  // turns out to be the coarsest ignores the lumping.
  numeric_lump(h, l, true);
  if (!h->side) h->side = side_stream(s);
  stream_after(h->side, s);
  numeric_damping(h, l, h->side, h->err + 2);
  L.nc = aggregate(n, nnzG, grp, gcol, o.agg_order, o.seed, l,
                   o.isolated == SA_ISOLATED_SINGLETON, L.agg, L.is_root, tmp, &root_vertex,
                   &L.mis_rounds, s);
  stream_after(s, h->side);
  if (nnzG == 0) {  // no strong connection: the coarsest level, which keeps no numeric part
    L.Abar = Csr{};
    L.invD = L.lam_d = L.omega_d = nullptr;
    return false;
  }
  if (L.nc >= n) throw Error(SA_ERR_COARSEN_STALLED, "coarsening stalled");
  int32_t ew[4];  // main word (lumping) and the damping word, in one readback
  readback(ew, h->err, sizeof(ew), s);
  if (ew[0] & E_ZERO_FDIAG)
    throw Error(SA_ERR_NONPOSITIVE_DIAG, "zero diagonal in the filtered matrix");
  if (ew[2] & E_LAMBDA) throw Error(SA_ERR_NEGATIVE_EIGENVALUE, "eigenvalue estimate not positive");
  numeric_prolong(h, l, true);
  return true;
}

// R_l = P_l^T and A_{l+1} = R_l (A_l P_l); P_1 first gets the nullspace scaling.  fresh:
// allocate level l+1; otherwise overwrite the values of R_l and A_{l+1}.
static bool resetup_plans_enabled() {
  const char *e = std::getenv("SAAMG_RESETUP_PLAN");
  return !(e && e[0] == '0');
}
static Csr keep_copy(const Csr &src, Arena &ar, hipStream_t s) {
  Csr d = src;
  d.rp = ar.alloc<int32_t>(src.n + 1);
  d.col = ar.alloc<int32_t>(src.nnz > 0 ? src.nnz : 1);
  d.val = ar.alloc<double>(src.nnz > 0 ? src.nnz : 1);
  d.bstart = nullptr;
  d.nblk = 0;
  SA_HIP(hipMemcpyAsync(d.rp, src.rp, sizeof(int32_t) * (src.n + 1), hipMemcpyDeviceToDevice, s));
  if (src.nnz > 0) {
    SA_HIP(hipMemcpyAsync(d.col, src.col, sizeof(int32_t) * src.nnz, hipMemcpyDeviceToDevice, s));
    SA_HIP(hipMemcpyAsync(d.val, src.val, sizeof(double) * src.nnz, hipMemcpyDeviceToDevice, s));
  }
  return d;
}

// A re-setup (fresh false) after the first takes the values of R, A P and A_{l+1} through the
// plans the first one built (R from P by the position map, each product entry summed over
// its list in Gustavson order): bitwise the values the full products give, without their
// symbolic passes.  SAAMG_RESETUP_PLAN=0 keeps the full products.
static void galerkin(sa_hierarchy *h, int l, bool fresh, const double *dB) {
  const hipStream_t s = h->stream;
  Level &L = h->lv[l];
  if (l == 0 && dB) scale_rows(L.P, dB, s);
  const bool plans = !fresh && resetup_plans_enabled();
  if (plans && L.planned) {
    transpose_values(L.P, L.rperm, L.R, s);
    spgemm_numeric(L.A, L.P, L.pap, L.APk, s);
    spgemm_numeric(L.R, L.APk, L.prap, h->lv[l + 1].A, s);
    return;
  }
  Arena tmp;
  tmp.stream = s;
  if (fresh) {
    transpose(L.P, h->ar, L.R, s);
    spmv_plan(L.R, h->ar, s);
  } else {
    Csr R;
    transpose(L.P, tmp, R, s);
    take_values(R, L.R, s);
  }
  Csr AP, Ac;
  spgemm(L.A, L.P, tmp, AP, s);
  if (fresh) {
    spgemm(L.R, AP, h->ar, Ac, s);
    spmv_plan(Ac, h->ar, s);
    double *cxyz = nullptr;  // coarse coordinates: the aggregates' centroids
    if (h->dim > 0) {
      cxyz = h->ar.alloc<double>((int64_t)L.nc * h->dim);
      aggregate_centroids(L.A.n / L.bs, L.agg, L.nc, L.xyz, h->dim, cxyz, s);
    }
    double *Bnext = L.Bc;
    h->lv.emplace_back();  // invalidates L
    h->lv[l + 1].A = Ac;
    h->lv[l + 1].As = Ac;
    h->lv[l + 1].xyz = cxyz;
    if (h->k > 0) {
      h->lv[l + 1].bs = h->k;
      h->lv[l + 1].B = Bnext;
    }
  } else {
    spgemm(L.R, AP, tmp, Ac, s);
    take_values(Ac, h->lv[l + 1].A, s);  // As shares A's arrays on coarse levels
    if (plans) {  // the first re-setup: keep A P and build the plans for the next ones
      L.APk = keep_copy(AP, h->ar, s);
      spgemm_plan(L.A, L.P, L.APk, h->ar, L.pap, h->err, E_PLAN, s);
      spgemm_plan(L.R, L.APk, h->lv[l + 1].A, h->ar, L.prap, h->err, E_PLAN, s);
      transpose_perm(L.P, L.R, h->ar, &L.rperm, s);
      check_err(h, E_PLAN, SA_ERR_INVALID_ARG, "re-setup plan: a product outside the pattern");
      L.planned = true;
    }
  }
}

// Scalars scattered over the levels, copied into one buffer for a single readback.
constexpr int kMaxGather = 48;  // 3 per level, at most 16 levels
struct ScalarGather {
  const double *p[kMaxGather];
  int32_t n;
};
__global__ void k_gather_scalars(ScalarGather g, double *out) {
  const int i = threadIdx.x;
  if (i < g.n) out[i] = g.p[i] ? *g.p[i] : 0.0;
}

// GPU part of level l's smoother set-up on stream s: the inverse diagonal of A_l and the
// power method for its largest eigenvalue (non-positive diagonals flag E_DIAG in *err).
static void smoother_gpu(sa_hierarchy *h, int l, bool fresh, hipStream_t s, int32_t *err) {
  Level &L = h->lv[l];
  Arena tmp;
  tmp.stream = s;
  double *dval = tmp.alloc<double>(L.A.n);
  find_diag(L.A.n, L.A.rp, L.A.col, L.A.val, dval, s);
  if (fresh && !L.sm_invD) {
    L.sm_invD = h->ar.alloc<double>(L.A.n);
    L.sm_lam_d = h->ar.alloc<double>(1);
  }
  inv_diag(L.A.n, dval, L.sm_invD, err, s);
  power_method(L.A, L.sm_invD, h->opt.power_iters, h->opt.seed, l, 1, L.sm_lam_d, s);
}

// Queues level l's smoother set-up on the side stream (level l is known not to be the
// coarsest): after the main stream's work so far (A_l, and any earlier use of blocks handed
// out below), with its own error word; finish_setup joins it.
static void smoother_async(sa_hierarchy *h, int l) {
  Level &L = h->lv[l];
  L.sm_invD = h->ar.alloc<double>(L.A.n);  // main-stream blocks: allocated before the wait
  L.sm_lam_d = h->ar.alloc<double>(1);
  if (!h->side) h->side = side_stream(h->stream);
  stream_after(h->side, h->stream);
  smoother_gpu(h, l, true, h->side, h->err + 1);
  L.sm_pending = true;
}

// Smoothers of every level but the coarsest, the coarsest level's dense inverse, the FP32
// copies and the solve workspace.  fresh: allocate; otherwise recompute in place.
static void finish_setup(sa_hierarchy *h, bool fresh) {
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  const int nl = (int)h->lv.size();
  const int32_t n = h->n;
  bool joined = false;
  for (int l = 0; l + 1 < nl; ++l) {
    Level &L = h->lv[l];
    if (!L.sm_pending) smoother_gpu(h, l, fresh, s, h->err);
    else if (!joined) {  // the levels queued on the side stream: join them once
      stream_after(s, h->side);
      joined = true;
    }
  }
  // the error words (main and side stream) and every level's eigenvalue and damping scalars
  // in two readbacks; the checks keep the level-by-level order
  int32_t ew[4];
  readback(ew, h->err, sizeof(ew), s);
  if ((ew[0] | ew[1]) & E_DIAG)
    throw Error(SA_ERR_NONPOSITIVE_DIAG, "non-positive diagonal in a level operator");
  std::vector<double> sc;
  if (nl > 1) {
    ScalarGather g{};
    for (int l = 0; l + 1 < nl; ++l) {
      g.p[3 * l] = h->lv[l].sm_lam_d;
      g.p[3 * l + 1] = h->lv[l].lam_d;
      g.p[3 * l + 2] = h->lv[l].lam_d ? h->lv[l].lam_d + 1 : nullptr;
    }
    g.n = 3 * (nl - 1);
    Arena tmp;
    tmp.stream = s;
    double *d = tmp.alloc<double>(g.n);
    k_gather_scalars<<<1, 64, 0, s>>>(g, d);
    SA_LAUNCH_CHECK();
    sc.resize(g.n);
    readback(sc.data(), d, sizeof(double) * g.n, s);
  }
  for (int l = 0; l + 1 < nl; ++l) {
    Level &L = h->lv[l];
    L.sm_pending = false;
    const double lam = sc[3 * l];
    if (!(lam > 0.0) || !std::isfinite(lam))
      throw Error(SA_ERR_NEGATIVE_EIGENVALUE, "smoother eigenvalue estimate not positive");
    L.sm_lam = lam * o.cheb_boost;
    chebyshev_scalars(L, o);
    if (L.lam_d) {
      L.lam = sc[3 * l + 1];
      L.omega = sc[3 * l + 2];
    }
  }
  Level &Lc = h->lv[nl - 1];
  if (Lc.A.n > kMaxDense)
    throw Error(SA_ERR_COARSE_FACTOR, "coarsest level too large for the dense solver");
  if (fresh) Lc.Ainv = h->ar.alloc<double>((int64_t)Lc.A.n * Lc.A.n);
  coarse_inverse(Lc.A, Lc.Ainv, h->err, o.coarse_solver == SA_COARSE_LU, s);
  check_err(h, E_ASYM, SA_ERR_COARSE_FACTOR,
            "coarsest operator not symmetric: use the LU coarse solver");
  check_err(h, E_CHOL, SA_ERR_COARSE_FACTOR,
            o.coarse_solver == SA_COARSE_LU ? "coarse LU pivot zero"
                                            : "coarse Cholesky pivot not positive");
  // FP32 copies of the hierarchy for the FP32 V-cycle
  const bool f32 = o.precision == SA_FP32_VCYCLE;
  for (int l = 0; l < nl; ++l) {
    Level &L = h->lv[l];
    const int32_t m = L.A.n;
    if (fresh) {
      L.f = h->ar.alloc<double>(m);
      L.u = h->ar.alloc<double>(m);
      L.r = h->ar.alloc<double>(m);
      L.d1 = h->ar.alloc<double>(m);
      L.d2 = h->ar.alloc<double>(m);
    }
    if (f32) {
      if (fresh) {
        L.ff = h->ar.alloc<float>(m);
        L.uf = h->ar.alloc<float>(m);
        L.rf = h->ar.alloc<float>(m);
        L.d1f = h->ar.alloc<float>(m);
        L.d2f = h->ar.alloc<float>(m);
      }
      if (l + 1 < nl) {
        if (fresh) {
          L.Af = h->ar.alloc<float>(L.A.nnz);
          L.Pf = h->ar.alloc<float>(L.P.nnz);
          L.Rf = h->ar.alloc<float>(L.R.nnz);
          L.sm_invDf = h->ar.alloc<float>(m);
        }
        cast_f64_to_f32(L.A.val, L.Af, L.A.nnz, s);
        cast_f64_to_f32(L.P.val, L.Pf, L.P.nnz, s);
        cast_f64_to_f32(L.R.val, L.Rf, L.R.nnz, s);
        cast_f64_to_f32(L.sm_invD, L.sm_invDf, m, s);
      }
    }
    // the solve's SpMVs on A: every level but a coarsest one with more than one level (its
    // dense solve takes no SpMV); level 0 also serves the Krylov method
    if (l + 1 < nl || l == 0) {
      if (fresh) sell_build(L.A, L.Aell, f32 && l + 1 < nl, h->ar, s);
      else sell_values(L.A, L.Aell, s);
    }
  }
  if (fresh) {
    h->x = h->ar.alloc<double>(n);
    h->r = h->ar.alloc<double>(n);
    h->z = h->ar.alloc<double>(n);
    h->p = h->ar.alloc<double>(n);
    h->q = h->ar.alloc<double>(n);
    h->zold = h->ar.alloc<double>(n);
    h->w = h->ar.alloc<double>(n);
    h->tmp64 = h->ar.alloc<double>(std::max<int64_t>(n, kMaxDense));
    h->dws = h->ar.alloc<double>(dot_ws_size(n));
    h->S = h->ar.alloc<PcgScalars>(1);
  }
  SA_HIP(hipStreamSynchronize(s));
}

// Nullspace: checks B (n values in `loc` memory); when some entry differs from 1, loads it
// into h->dB and sets As = D_B A D_B on level 0, otherwise As = A.  Returns h->dB or null.
static double *apply_nullspace(sa_hierarchy *h, const double *B, sa_location loc) {
  const hipStream_t s = h->stream;
  const int32_t n = h->n;
  Level &L0 = h->lv[0];
  L0.As = L0.A;
  if (!B) return nullptr;
  std::vector<double> hb(n);
  SA_HIP(hipMemcpyAsync(hb.data(), B, sizeof(double) * n,
                        loc == SA_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, s));
  SA_HIP(hipStreamSynchronize(s));
  bool scaled = false;
  for (double v : hb) {
    if (!(v != 0.0) || !std::isfinite(v))
      throw Error(SA_ERR_INVALID_ARG, "nullspace entry zero or non-finite");
    if (v != 1.0) scaled = true;
  }
  if (!scaled) return nullptr;
  if (!h->dB) h->dB = h->ar.alloc<double>(n);
  if (!h->As0) h->As0 = h->ar.alloc<double>(L0.A.nnz);
  SA_HIP(hipMemcpyAsync(h->dB, hb.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  L0.As.val = h->As0;
  scale_sym(n, L0.A.rp, L0.A.col, L0.A.val, h->dB, L0.As.val, s);
  SA_HIP(hipStreamSynchronize(s));  // hb goes out of scope
  return h->dB;
}

// The input matrix's structure and values, one readback: row pointers spanning [0, nnz]
// first, then values, columns and diagonals.
static void validate_values(sa_hierarchy *h) {
  Level &L0 = h->lv[0];
  validate_csr(h->n, L0.A.nnz, L0.A.rp, L0.A.col, L0.A.val, h->err, h->stream);
  const int32_t e = read_err(h);
  if (e & E_SPAN) throw Error(SA_ERR_BAD_CSR, "row pointers do not span nnz");
  if (e & E_NONFINITE) throw Error(SA_ERR_INVALID_ARG, "non-finite matrix value");
  if (e & E_STRUCT) throw Error(SA_ERR_BAD_CSR, "columns out of range or not ascending");
  if (e & E_NODIAG) throw Error(SA_ERR_BAD_CSR, "missing diagonal");
}

static void setup_impl(sa_hierarchy *h, const sa_csr *A, const double *B,
                       const double *coords, int32_t dim, int32_t bs = 1,
                       const double *Bm = nullptr, int32_t k = 0) {
  const double t0 = now_s();
  const hipStream_t s = h->stream;
  sa_options &o = h->opt;
  validate_options(o);
  if (!A || A->n < 0 || A->nnz < 0 || A->nnz >= (int64_t)INT32_MAX || !A->row_ptr ||
      (A->nnz > 0 && (!A->col || !A->val)))
    throw Error(SA_ERR_INVALID_ARG, "bad matrix argument");
  if (A->n == 0) throw Error(SA_ERR_INVALID_ARG, "empty matrix");
  const int32_t n = A->n;
  h->n = n;
  h->err = h->ar.alloc<int32_t>(4);
  fill_i32(h->err, 0, 4, s);
  h->lv.emplace_back();
  Level &L0 = h->lv[0];
  L0.A.n = L0.A.ncols = n;
  L0.A.nnz = A->nnz;
  L0.A.rp = h->ar.alloc<int32_t>(n + 1);
  L0.A.col = h->ar.alloc<int32_t>(A->nnz);
  L0.A.val = h->ar.alloc<double>(A->nnz);
  copy_in(L0.A.rp, A->row_ptr, sizeof(int32_t) * (n + 1), A->loc, s);
  copy_in(L0.A.col, A->col, sizeof(int32_t) * A->nnz, A->loc, s);
  copy_in(L0.A.val, A->val, sizeof(double) * A->nnz, A->loc, s);
  validate_values(h);
  if (k > 0) {  // systems SA
    if (bs < 1 || bs > 16 || n % bs != 0)
      throw Error(SA_ERR_INVALID_ARG, "block size not in 1..16 or not dividing n");
    if (k > 16) throw Error(SA_ERR_INVALID_ARG, "nullspace dimension not in 1..16");
    if (o.variants & (SA_SPRSFY | SA_CNSTRNT))
      throw Error(SA_ERR_INVALID_ARG, "Sprsfy and Cnstrnt are not defined for systems");
    h->k = k;
    L0.bs = bs;
    L0.B = h->ar.alloc<double>((int64_t)n * k);
    copy_in(L0.B, Bm, sizeof(double) * (size_t)n * k, A->loc, s);
    check_finite(L0.B, (int64_t)n * k, h->err, E_NONFINITE, s);
    check_err(h, E_NONFINITE, SA_ERR_INVALID_ARG, "non-finite nullspace entry");
  }
  if (coords) {
    const int64_t npts = n / L0.bs;  // coordinates are per node
    if (dim < 1 || dim > 3) throw Error(SA_ERR_INVALID_ARG, "coordinate dimension not 1..3");
    h->dim = dim;
    L0.xyz = h->ar.alloc<double>(npts * dim);
    copy_in(L0.xyz, coords, sizeof(double) * npts * dim, A->loc, s);
    check_finite(L0.xyz, npts * dim, h->err, E_COORD, s);
    check_err(h, E_COORD, SA_ERR_INVALID_ARG, "non-finite coordinate");
  }
  spmv_plan(L0.A, h->ar, s);
  const double *dB = apply_nullspace(h, B, A->loc);
  for (int l = 0;; ++l) {
    if (h->lv[l].A.n <= o.max_coarse || l + 1 >= o.max_levels) break;
    if (!build_level(h, l)) {
      Level &Lc = h->lv[l];
      Lc.nc = 0;
      Lc.mask = nullptr;
      Lc.agg = nullptr;
      Lc.is_root = nullptr;
      break;
    }
    smoother_async(h, l);  // overlaps the Galerkin product and the next levels
    galerkin(h, l, true, dB);
  }
  finish_setup(h, true);
  h->setup_seconds = now_s() - t0;
}

// New values on the setup's pattern: every symbolic decision is kept (strength labels and
// Sprsfy drops, aggregates, the patterns of the filtered matrices, P, R and every A_l) and
// the numbers are recomputed in the setup's order, each into the existing arrays.
static void resetup_impl(sa_hierarchy *h, const double *val, const double *B, sa_location loc) {
  if (h->k > 0 && B) throw Error(SA_ERR_INVALID_ARG, "a systems hierarchy keeps its nullspace");
  const double t0 = now_s();
  const hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  h->valid = false;
  fill_i32(h->err, 0, 4, s);
  copy_in(L0.A.val, val, sizeof(double) * L0.A.nnz, loc, s);
  validate_values(h);
  const double *dB = apply_nullspace(h, B, loc);
  const int nl = (int)h->lv.size();
  for (int l = 0; l + 1 < nl; ++l) {
    numeric_level(h, l, false);
    galerkin(h, l, false, dB);
  }
  finish_setup(h, false);
  h->setup_seconds = now_s() - t0;
  h->valid = true;
}

// ---- fine-level SpMV timing ------------------------------------------------------------------
static void prof_begin(sa_hierarchy *h, int l) {
  if (!h->prof || l != 0) return;
  if (h->nev + 2 > (int32_t)h->ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      SA_HIP(hipEventCreate(&e));
      h->ev.push_back(e);
    }
    h->ev_bytes.resize(h->ev.size() / 2);
  }
  SA_HIP(hipEventRecord(h->ev[h->nev], h->stream));
}
// `vec` = number of n-vectors the launch's epilogue and input read or write (x included).
// Algorithmic bytes: the entries (index + value; sliced-ELL padding not counted), the row
// structure the kernel reads (row pointers, or slice offsets) and the vectors.
static void prof_end(sa_hierarchy *h, int l, int vec, int elem) {
  if (!h->prof || l != 0) return;
  SA_HIP(hipEventRecord(h->ev[h->nev + 1], h->stream));
  const Csr &A = h->lv[0].A;
  const Sell &S = h->lv[0].Aell;
  const double rows = S.ptr ? 4.0 * (S.nslice + 1) : 4.0 * (A.n + 1);
  h->ev_bytes[h->nev / 2] = (double)A.nnz * (4 + elem) + rows + (double)vec * elem * A.n;
  h->nev += 2;
}
// After a synchronisation: fold the recorded pairs into the totals.
static void prof_collect(sa_hierarchy *h) {
  if (!h->prof) return;
  for (int32_t k = 0; k < h->nev; k += 2) {
    float ms = 0.f;
    SA_HIP(hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]));
    h->prof_ms += ms;
    h->prof_bytes += h->ev_bytes[k / 2];
    ++h->prof_launches;
  }
  h->nev = 0;
}

// ---- V-cycle ---------------------------------------------------------------------------------
template <class T>
struct LevelView {
  SpmvArgs<T> A, P, R;
  const T *invD;
  T *f, *u, *r, *d1, *d2;
};

static LevelView<double> view64(Level &L) {
  LevelView<double> v;
  v.A = with_sell(spmv_args<double>(L.A, L.A.val, nullptr), L.Aell, L.Aell.val);
  v.P = spmv_args<double>(L.P, L.P.val, nullptr);
  v.R = spmv_args<double>(L.R, L.R.val, nullptr);
  v.invD = L.sm_invD;
  v.f = L.f;
  v.u = L.u;
  v.r = L.r;
  v.d1 = L.d1;
  v.d2 = L.d2;
  return v;
}
static LevelView<float> view32(Level &L) {
  LevelView<float> v;
  v.A = with_sell(spmv_args<float>(L.A, L.Af, nullptr), L.Aell, (const float *)L.Aell.valf);
  v.P = spmv_args<float>(L.P, L.Pf, nullptr);
  v.R = spmv_args<float>(L.R, L.Rf, nullptr);
  v.invD = L.sm_invDf;
  v.f = L.ff;
  v.u = L.uf;
  v.r = L.rf;
  v.d1 = L.d1f;
  v.d2 = L.d2f;
  return v;
}

template <class T>
static void smooth(sa_hierarchy *h, int l, Level &L, LevelView<T> &v, const T *f, T *u,
                   bool uzero) {
  const int es = (int)sizeof(T);
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  const int32_t n = L.A.n;
  SpmvArgs<T> A = v.A;
  if (o.smoother == SA_JACOBI) {
    const T w = (T)L.jac_w;
    int sweep = 0;
    if (uzero) {
      jacobi_first<T>(n, f, v.invD, w, u, s);
      sweep = 1;
    }
    for (; sweep < o.degree; ++sweep) {
      A.x = u;
      prof_begin(h, l);
      spmv_jacobi<T>(A, f, v.invD, w, v.d1, s);
      prof_end(h, l, 4, es);
      SA_HIP(hipMemcpyAsync(u, v.d1, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    }
    return;
  }
  const T theta = (T)L.cheb_theta;
  T *dc = v.d1, *dn = v.d2;
  const T *rin;
  if (uzero) {
    cheb_first<T>(n, f, v.invD, theta, dc, u, o.degree == 1, s);
    rin = f;
  } else {
    A.x = u;
    prof_begin(h, l);
    spmv_cheb_start<T>(A, f, v.invD, theta, v.r, dc, s);
    prof_end(h, l, 5, es);
    if (o.degree == 1) vec_add<T>(n, u, dc, s);
    rin = v.r;
  }
  for (int m = 1; m < o.degree; ++m) {
    A.x = dc;
    const bool last = (m == o.degree - 1);
    prof_begin(h, l);
    spmv_cheb_step<T>(A, rin, v.r, v.invD, (T)L.cheb_c1[m - 1], (T)L.cheb_c2[m - 1], u,
                      uzero && m == 1, dn, last, s);
    // x = d, rin, invD, rout, u (read unless from zero), u written, dout unless last
    prof_end(h, l, 5 + ((uzero && m == 1) ? 0 : 1) + (last ? 0 : 1), es);
    rin = v.r;
    std::swap(dc, dn);
  }
}

template <class T>
static void coarse_apply(sa_hierarchy *h, Level &L, const T *f, T *u);
template <>
void coarse_apply<double>(sa_hierarchy *h, Level &L, const double *f, double *u) {
  gemv_f64(L.A.n, L.Ainv, f, u, h->stream);
}
template <>
void coarse_apply<float>(sa_hierarchy *h, Level &L, const float *f, float *u) {
  double *f64 = h->tmp64;
  double *u64 = L.u;
  cast_f32_to_f64(f, f64, L.A.n, h->stream);
  gemv_f64(L.A.n, L.Ainv, f64, u64, h->stream);
  cast_f64_to_f32(u64, u, L.A.n, h->stream);
}

template <class T>
static void vcycle(sa_hierarchy *h, int l, const T *f, T *u) {
  Level &L = h->lv[l];
  const int nl = (int)h->lv.size();
  if (l + 1 == nl) {
    coarse_apply<T>(h, L, f, u);
    return;
  }
  LevelView<T> v;
  if constexpr (sizeof(T) == 8) v = view64(L);
  else v = view32(L);
  LevelView<T> vc;
  if constexpr (sizeof(T) == 8) vc = view64(h->lv[l + 1]);
  else vc = view32(h->lv[l + 1]);
  const hipStream_t s = h->stream;
  smooth<T>(h, l, L, v, f, u, true);
  SpmvArgs<T> A = v.A;
  A.x = u;
  prof_begin(h, l);
  spmv_resid<T>(A, f, v.r, s);
  prof_end(h, l, 3, (int)sizeof(T));
  SpmvArgs<T> R = v.R;
  R.x = v.r;
  spmv_store<T>(R, vc.f, s);
  vcycle<T>(h, l + 1, vc.f, vc.u);
  SpmvArgs<T> P = v.P;
  P.x = vc.u;
  spmv_add<T>(P, u, s);
  smooth<T>(h, l, L, v, f, u, false);
}

// z = M^{-1} r at the fine level, in the hierarchy's precision.
static void precondition(sa_hierarchy *h, const double *r, double *z) {
  Level &L0 = h->lv[0];
  if (h->opt.precision == SA_FP32_VCYCLE && h->lv.size() > 1) {
    cast_f64_to_f32(r, L0.ff, h->n, h->stream);
    vcycle<float>(h, 0, L0.ff, L0.uf);
    cast_f32_to_f64(L0.uf, z, h->n, h->stream);
  } else {
    vcycle<double>(h, 0, r, z);
  }
}

static sa_status solve_impl(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                            int32_t *iterations, double *relres) {
  if (!h->valid) throw Error(SA_ERR_INVALID_ARG, "hierarchy left unusable by a failed re-setup");
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  const int32_t n = h->n;
  const bool pr = (o.pcg_beta == SA_BETA_PR) ||
                  (o.pcg_beta < 0 && o.precision == SA_FP32_VCYCLE);
  copy_in(h->r, b, sizeof(double) * n, loc, s);
  fill_f64(h->x, 0.0, n, s);
  PcgScalars *S = h->S;
  SA_HIP(hipMemsetAsync(S, 0, sizeof(PcgScalars), s));
  dot_f64(h->r, h->r, n, &S->rr, h->dws, s);
  const double g0 = read1(&S->rr, s);
  int32_t its = 0;
  double rr = g0;
  sa_status st = SA_NOT_CONVERGED;
  auto finish = [&]() {
    if (loc == SA_DEVICE)
      SA_HIP(hipMemcpyAsync(x, h->x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    else
      SA_HIP(hipMemcpyAsync(x, h->x, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
  };
  if (!std::isfinite(g0)) throw Error(SA_ERR_INVALID_ARG, "non-finite right-hand side");
  if (g0 == 0.0) {
    finish();
    if (iterations) *iterations = 0;
    if (relres) *relres = 0.0;
    return SA_OK;
  }
  const double thr = (o.rtol * o.rtol) * g0;
  precondition(h, h->r, h->z);
  SA_HIP(hipMemcpyAsync(h->p, h->z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  dot_f64(h->r, h->z, n, &S->rho1, h->dws, s);
  pcg_init_rho(S, s);
  SpmvArgs<double> A =
      with_sell(spmv_args<double>(h->lv[0].A, h->lv[0].A.val, h->p), h->lv[0].Aell,
                h->lv[0].Aell.val);
  for (int32_t k = 1; k <= o.max_iter; ++k) {
    prof_begin(h, 0);
    spmv_store<double>(A, h->q, s);
    prof_end(h, 0, 2, 8);
    dot_f64(h->p, h->q, n, &S->pq, h->dws, s);
    pcg_alpha(S, s);
    pcg_update_xr(n, h->x, h->r, h->p, h->q, S, s);
    dot_f64(h->r, h->r, n, &S->rr, h->dws, s);
    PcgScalars hs;
    readback(&hs, S, sizeof(PcgScalars), s);
    prof_collect(h);
    if (hs.err) return SA_ERR_BREAKDOWN;
    rr = hs.rr;
    its = k;
    if (rr <= thr) {
      st = SA_OK;
      break;
    }
    if (pr) SA_HIP(hipMemcpyAsync(h->zold, h->z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    precondition(h, h->r, h->z);
    dot_f64(h->r, h->z, n, &S->rho1, h->dws, s);
    if (pr) {
      vec_sub(n, h->z, h->zold, h->w, s);
      dot_f64(h->r, h->w, n, &S->rw, h->dws, s);
    }
    pcg_beta(S, pr, s);
    pcg_update_p(n, h->p, h->z, S, s);
  }
  if (st != SA_OK) {
    PcgScalars hs;
    readback(&hs, S, sizeof(PcgScalars), s);
    if (hs.err) return SA_ERR_BREAKDOWN;
    its = o.max_iter;
  }
  finish();
  prof_collect(h);
  if (iterations) *iterations = its;
  if (relres) *relres = std::sqrt(rr / g0);
  return st;
}

// GMRES workspace for n unknowns and restart m, carved from one block in this order, each
// part starting on a 256-byte boundary: V ((m+1) n), Z (m n), H ((m+1) m), cs, sn (m), g
// (m+1), y (m), c (m+1), the inner-product partials ((m+1) dot_ws_size(n)), the scalars.
static size_t gmres_part(int64_t count, size_t elem) {
  return ((size_t)(count > 0 ? count : 1) * elem + 255) & ~(size_t)255;
}
size_t gmres_work_bytes(int32_t n, int32_t m) {
  const int64_t N = n, M = m;
  return gmres_part((M + 1) * N, 8) + gmres_part(M * N, 8) + gmres_part((M + 1) * M, 8) +
         2 * gmres_part(M, 8) + gmres_part(M + 1, 8) + gmres_part(M, 8) +
         gmres_part(M + 1, 8) + gmres_part((M + 1) * dot_ws_size(N), 8) +
         gmres_part(1, sizeof(GmresScalars));
}
GmresWork gmres_work_carve(void *base, int32_t n, int32_t m) {
  const int64_t N = n, M = m;
  char *p = (char *)base;
  auto take = [&](int64_t count, size_t elem) {
    char *q = p;
    p += gmres_part(count, elem);
    return q;
  };
  GmresWork w;
  w.V = (double *)take((M + 1) * N, 8);
  w.Z = (double *)take(M * N, 8);
  w.H = (double *)take((M + 1) * M, 8);
  w.cs = (double *)take(M, 8);
  w.sn = (double *)take(M, 8);
  w.g = (double *)take(M + 1, 8);
  w.y = (double *)take(M, 8);
  w.c = (double *)take(M + 1, 8);
  w.ws = (double *)take((M + 1) * dot_ws_size(N), 8);
  w.S = (GmresScalars *)take(1, sizeof(GmresScalars));
  return w;
}

// Restarted flexible GMRES(m), the V-cycle as right preconditioner (the paper's solver for
// its nonsymmetric wind-turbine systems, Sec. 3.4).  x0 = 0; Arnoldi by classical
// Gram-Schmidt applied twice; Givens rotations; stop when the least-squares residual
// |g_{j+1}| <= rtol ||b||; at a restart the true residual b - A x is formed and tested; a zero
// new basis norm ends the cycle with the exact Krylov solution.  The flexible form keeps the
// preconditioned vectors Z and updates x += Z y.  Iterations count Arnoldi steps.
// The workspace comes from the caller (gmres_work_carve).  direct_reads: the scalars are read
// back by a plain copy into host memory instead of through the pinned staging buffer, which
// may be allocated on a thread's first use.
sa_status gmres_run(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                    int32_t restart, const GmresWork &wk, bool direct_reads,
                    int32_t *iterations, double *relres) {
  if (!h->valid) throw Error(SA_ERR_INVALID_ARG, "hierarchy left unusable by a failed re-setup");
  if (restart < 1 || restart > kMaxRestart) throw Error(SA_ERR_INVALID_ARG, "restart not in 1..1024");
  const hipStream_t s = h->stream;
  const sa_options &o = h->opt;
  const int32_t n = h->n;
  const int32_t m = restart;
  double *V = wk.V, *Z = wk.Z, *H = wk.H, *cs = wk.cs, *sn = wk.sn, *g = wk.g, *y = wk.y,
         *c = wk.c, *ws = wk.ws;
  GmresScalars *S = wk.S;
  auto read_scalars = [&](GmresScalars *hs) {
    if (direct_reads) {
      SA_HIP(hipMemcpyAsync(hs, S, sizeof(GmresScalars), hipMemcpyDeviceToHost, s));
      SA_HIP(hipStreamSynchronize(s));
    } else {
      readback(hs, S, sizeof(GmresScalars), s);
    }
  };
  static_assert(sizeof(GmresScalars) % 4 == 0, "scalars cleared as 32-bit words");
  fill_i32((int32_t *)S, 0, (int64_t)(sizeof(GmresScalars) / 4), s);
  double *r = h->r, *xv = h->x, *bd = h->q;
  copy_in(bd, b, sizeof(double) * n, loc, s);
  SA_HIP(hipMemcpyAsync(r, bd, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  fill_f64(xv, 0.0, n, s);
  dot_f64(r, r, n, &S->nrm2, h->dws, s);
  gmres_start(S, r, V, n, g, s);  // beta = ||b||, v_0 = b / beta
  GmresScalars hs;
  read_scalars(&hs);
  const double bn = hs.beta;
  auto finish = [&]() {
    SA_HIP(hipMemcpyAsync(x, xv, sizeof(double) * n,
                          loc == SA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
  };
  if (!std::isfinite(bn)) throw Error(SA_ERR_INVALID_ARG, "non-finite right-hand side");
  if (bn == 0.0) {
    finish();
    if (iterations) *iterations = 0;
    if (relres) *relres = 0.0;
    return SA_OK;
  }
  const double target = o.rtol * bn;
  SpmvArgs<double> A =
      with_sell(spmv_args<double>(h->lv[0].A, h->lv[0].A.val, nullptr), h->lv[0].Aell,
                h->lv[0].Aell.val);
  double res = bn;
  int32_t total = 0;
  bool converged = false;
  for (;;) {
    int32_t kdim = 0;
    for (int32_t j = 0; j < m && total < o.max_iter; ++j) {
      double *vj = V + (int64_t)j * n, *zj = Z + (int64_t)j * n, *w = V + (int64_t)(j + 1) * n;
      precondition(h, vj, zj);
      A.x = zj;
      prof_begin(h, 0);
      spmv_store<double>(A, w, s);
      prof_end(h, 0, 2, 8);
      for (int32_t pass = 0; pass < 2; ++pass) {
        multi_dot_f64(V, n, j + 1, w, n, c, ws, s);
        multi_axpy_f64(V, n, j + 1, c, w, n, false, s);
        gmres_accum(H, m, j, c, pass, s);
      }
      dot_f64(w, w, n, &S->hn2, h->dws, s);
      gmres_normalize(S, H, m, j, w, w, n, s);
      gmres_givens(H, m, j, cs, sn, g, S, s);
      read_scalars(&hs);
      prof_collect(h);
      ++total;
      kdim = j + 1;
      res = hs.res;
      if (!std::isfinite(res)) return SA_ERR_BREAKDOWN;
      if (res <= target || hs.hn == 0.0) {
        converged = true;
        break;
      }
    }
    if (kdim == 0) break;
    gmres_backsolve(H, m, kdim, g, y, S, s);
    multi_axpy_f64(Z, n, kdim, y, xv, n, true, s);
    read_scalars(&hs);
    if (hs.err) return SA_ERR_BREAKDOWN;
    if (converged || total >= o.max_iter) break;
    // restart from the true residual
    A.x = xv;
    spmv_resid<double>(A, bd, r, s);
    dot_f64(r, r, n, &S->nrm2, h->dws, s);
    gmres_start(S, r, V, n, g, s);
    read_scalars(&hs);
    res = hs.beta;
    if (res <= target) {
      converged = true;
      break;
    }
  }
  finish();
  prof_collect(h);
  if (iterations) *iterations = total;
  if (relres) *relres = res / bn;
  return converged ? SA_OK : SA_NOT_CONVERGED;
}

// GMRES with its workspace taken from the library's device-memory cache for the call.
static sa_status gmres_impl(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                            int32_t restart, int32_t *iterations, double *relres) {
  if (restart < 1 || restart > kMaxRestart) throw Error(SA_ERR_INVALID_ARG, "restart not in 1..1024");
  Arena tmp;
  tmp.stream = h->stream;
  void *base = tmp.alloc<unsigned char>((int64_t)gmres_work_bytes(h->n, restart));
  return gmres_run(h, b, x, loc, restart, gmres_work_carve(base, h->n, restart), false,
                   iterations, relres);
}

template <class F>
static sa_status guarded(F &&fn) {
  try {
    return fn();
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SA_ERR_OOM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return SA_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown failure";
    return SA_ERR_HIP;
  }
}

}  // namespace sa

namespace sa {
// Frees a hierarchy whose stream has no pending work that uses it, without synchronising
// that stream (its blocks return to the stream's cache).
void hierarchy_release_nosync(sa_hierarchy *h) {
  if (!h) return;
  h->ar.release();
  delete h;
}
}  // namespace sa

using namespace sa;

extern "C" {

void sa_default_options(sa_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(sa_options);
  o->variants = 0;
  o->theta = 0.02;
  o->tau = 1.1;
  o->sigma = 1.0 / 3.0;
  o->one_norm_power = 0;
  o->power_iters = 10;
  o->seed = 12345;
  o->agg_order = SA_AGG_NATURAL;
  o->max_levels = 10;
  o->max_coarse = 1000;
  o->smoother = SA_CHEBYSHEV;
  o->degree = 2;
  o->precision = SA_FP64;
  o->cheb_ratio = 10.0;
  o->cheb_boost = 1.0;
  o->rtol = 1e-8;
  o->max_iter = 500;
  o->pcg_beta = -1;
  o->dist_power = 1;
  o->coarse_solver = SA_COARSE_CHOLESKY;
  o->isolated = SA_ISOLATED_LEFT_OUT;
}

sa_status sa_setup_coords(const sa_context *ctx, const sa_csr *A, const double *nullspace,
                          const double *coords, int32_t dim, const sa_options *o,
                          sa_hierarchy **out) {
  if (!out) return SA_ERR_INVALID_ARG;
  *out = nullptr;
  return guarded([&]() -> sa_status {
    std::unique_ptr<sa_hierarchy> h(new sa_hierarchy());
    h->stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    h->ar.stream = h->stream;
    if (o) h->opt = *o;
    else sa_default_options(&h->opt);
    try {
      setup_impl(h.get(), A, nullspace, coords, dim);
    } catch (...) {
      (void)hipStreamSynchronize(h->stream);
      if (h->side) (void)hipStreamSynchronize(h->side);
      throw;
    }
    *out = h.release();
    return SA_OK;
  });
}

sa_status sa_setup(const sa_context *ctx, const sa_csr *A, const double *nullspace,
                   const sa_options *o, sa_hierarchy **out) {
  return sa_setup_coords(ctx, A, nullspace, nullptr, 0, o, out);
}

sa_status sa_setup_system(const sa_context *ctx, const sa_csr *A, int32_t block_size,
                          const double *nullspace, int32_t k, const double *coords, int32_t dim,
                          const sa_options *o, sa_hierarchy **out) {
  if (!out) return SA_ERR_INVALID_ARG;
  *out = nullptr;
  if (!nullspace || k < 1) return SA_ERR_INVALID_ARG;
  return guarded([&]() -> sa_status {
    std::unique_ptr<sa_hierarchy> h(new sa_hierarchy());
    h->stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    h->ar.stream = h->stream;
    if (o) h->opt = *o;
    else sa_default_options(&h->opt);
    try {
      setup_impl(h.get(), A, nullptr, coords, dim, block_size, nullspace, k);
    } catch (...) {
      (void)hipStreamSynchronize(h->stream);
      if (h->side) (void)hipStreamSynchronize(h->side);
      throw;
    }
    *out = h.release();
    return SA_OK;
  });
}

sa_status sa_resetup(sa_hierarchy *h, const double *val, const double *nullspace,
                     sa_location loc) {
  if (!h || !val || h->lv.empty()) return SA_ERR_INVALID_ARG;
  return guarded([&]() -> sa_status {
    try {
      resetup_impl(h, val, nullspace, loc);
    } catch (...) {
      (void)hipStreamSynchronize(h->stream);
      throw;
    }
    return SA_OK;
  });
}

sa_status sa_solve(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                   int32_t *iterations, double *rel_residual) {
  if (!h || !b || !x) return SA_ERR_INVALID_ARG;
  return guarded([&]() -> sa_status {
    sa_status st = solve_impl(h, b, x, loc, iterations, rel_residual);
    if (st < 0) {
      (void)hipStreamSynchronize(h->stream);
      g_last_error = "CG breakdown (p'Ap <= 0 or r'z <= 0)";
    }
    return st;
  });
}

sa_status sa_solve_gmres(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                         int32_t restart, int32_t *iterations, double *rel_residual) {
  if (!h || !b || !x) return SA_ERR_INVALID_ARG;
  return guarded([&]() -> sa_status {
    sa_status st = gmres_impl(h, b, x, loc, restart, iterations, rel_residual);
    if (st < 0) {
      (void)hipStreamSynchronize(h->stream);
      g_last_error = "GMRES breakdown (non-finite residual or singular least-squares system)";
    }
    return st;
  });
}

sa_status sa_vcycle(sa_hierarchy *h, const double *f, double *z) {
  if (!h || !f || !z) return SA_ERR_INVALID_ARG;
  return guarded([&]() -> sa_status {
    precondition(h, f, z);
    SA_HIP(hipStreamSynchronize(h->stream));
    return SA_OK;
  });
}

sa_status sa_hierarchy_info(const sa_hierarchy *h, sa_info *info) {
  if (!h || !info) return SA_ERR_INVALID_ARG;
  std::memset(info, 0, sizeof(*info));
  info->levels = (int32_t)h->lv.size();
  double tot = 0.0;
  for (size_t l = 0; l < h->lv.size() && l < 16; ++l) {
    const Level &L = h->lv[l];
    info->n[l] = L.A.n;
    info->nnz[l] = L.A.nnz;
    info->nnz_p[l] = (l + 1 < h->lv.size()) ? L.P.nnz : 0;
    info->lambda[l] = L.lam;
    info->omega[l] = L.omega;
    info->smoother_lambda[l] = L.sm_lam;
    info->mis_rounds[l] = L.mis_rounds;
    tot += (double)L.A.nnz;
  }
  info->operator_complexity = tot / (double)h->lv[0].A.nnz;
  info->device_bytes = h->ar.bytes;
  info->setup_seconds = h->setup_seconds;
  return SA_OK;
}

static bool part_info(const sa_hierarchy *h, int32_t level, sa_part what, const void **ptr,
                      int64_t *count, int *esize) {
  if (!h || level < 0 || level >= (int32_t)h->lv.size()) return false;
  const Level &L = h->lv[level];
  const bool has_p = level + 1 < (int32_t)h->lv.size();
  *ptr = nullptr;
  *count = 0;
  *esize = 4;
  switch (what) {
    case SA_PART_A_RP: *ptr = L.A.rp; *count = L.A.n + 1; break;
    case SA_PART_A_COL: *ptr = L.A.col; *count = L.A.nnz; break;
    case SA_PART_A_VAL: *ptr = L.A.val; *count = L.A.nnz; *esize = 8; break;
    case SA_PART_MASK: *ptr = L.mask; *count = L.mask ? L.A.nnz : 0; *esize = 1; break;
    case SA_PART_AGG: *ptr = L.agg; *count = L.agg ? L.A.n / L.bs : 0; break;
    case SA_PART_ROOT: *ptr = L.is_root; *count = L.is_root ? L.A.n / L.bs : 0; *esize = 1; break;
    case SA_PART_ABAR_RP: *ptr = L.Abar.rp; *count = has_p ? L.Abar.n + 1 : 0; break;
    case SA_PART_ABAR_COL: *ptr = L.Abar.col; *count = has_p ? L.Abar.nnz : 0; break;
    case SA_PART_ABAR_VAL: *ptr = L.Abar.val; *count = has_p ? L.Abar.nnz : 0; *esize = 8; break;
    case SA_PART_INVD: *ptr = L.invD; *count = has_p ? L.A.n : 0; *esize = 8; break;
    case SA_PART_P_RP: *ptr = L.P.rp; *count = has_p ? L.P.n + 1 : 0; break;
    case SA_PART_P_COL: *ptr = L.P.col; *count = has_p ? L.P.nnz : 0; break;
    case SA_PART_P_VAL: *ptr = L.P.val; *count = has_p ? L.P.nnz : 0; *esize = 8; break;
    case SA_PART_R_RP: *ptr = L.R.rp; *count = has_p ? L.R.n + 1 : 0; break;
    case SA_PART_R_COL: *ptr = L.R.col; *count = has_p ? L.R.nnz : 0; break;
    case SA_PART_R_VAL: *ptr = L.R.val; *count = has_p ? L.R.nnz : 0; *esize = 8; break;
    case SA_PART_SM_INVD: *ptr = L.sm_invD; *count = has_p ? L.A.n : 0; *esize = 8; break;
    case SA_PART_PT_RP: *ptr = L.Pt.rp; *count = has_p && L.Pt.rp ? L.A.n + 1 : 0; break;
    case SA_PART_PT_COL: *ptr = L.Pt.col; *count = has_p ? L.Pt.nnz : 0; break;
    case SA_PART_PT_VAL: *ptr = L.Pt.val; *count = has_p ? L.Pt.nnz : 0; *esize = 8; break;
    case SA_PART_NULLSPACE: *ptr = L.B; *count = (int64_t)L.A.n * h->k; *esize = 8; break;
    case SA_PART_NODE_MASK: *ptr = L.nmask; *count = has_p ? L.Gn.nnz : 0; *esize = 1; break;
    case SA_PART_NODE_RP: *ptr = L.Gn.rp; *count = has_p && L.Gn.rp ? L.Gn.n + 1 : 0; break;
    case SA_PART_NODE_COL: *ptr = L.Gn.col; *count = has_p ? L.Gn.nnz : 0; break;
    case SA_PART_COORDS:
      *ptr = L.xyz;
      *count = (int64_t)(L.A.n / L.bs) * h->dim;  // one point per node
      *esize = 8;
      break;
    case SA_PART_COARSE_INV:
      *ptr = L.Ainv;
      *count = has_p ? 0 : (int64_t)L.A.n * L.A.n;
      *esize = 8;
      break;
    default: return false;
  }
  if (!*ptr) *count = 0;
  return true;
}

sa_status sa_export_size(const sa_hierarchy *h, int32_t level, sa_part what, int64_t *count) {
  const void *p;
  int es;
  if (!count || !part_info(h, level, what, &p, count, &es)) return SA_ERR_INVALID_ARG;
  return SA_OK;
}

sa_status sa_export_level(const sa_hierarchy *h, int32_t level, sa_part what, void *host_buf,
                          size_t bytes) {
  return guarded([&]() -> sa_status {
    const void *p;
    int64_t count;
    int es;
    if (!part_info(h, level, what, &p, &count, &es)) return SA_ERR_INVALID_ARG;
    if ((size_t)count * es > bytes || (count > 0 && !host_buf)) return SA_ERR_INVALID_ARG;
    if (count > 0) {
      SA_HIP(hipMemcpyAsync(host_buf, p, (size_t)count * es, hipMemcpyDeviceToHost, h->stream));
      SA_HIP(hipStreamSynchronize(h->stream));
    }
    return SA_OK;
  });
}

sa_status sa_profile_enable(sa_hierarchy *h, int32_t on) {
  if (!h) return SA_ERR_INVALID_ARG;
  return guarded([&]() -> sa_status {
    SA_HIP(hipStreamSynchronize(h->stream));
    prof_collect(h);
    h->prof = on != 0;
    h->prof_launches = 0;
    h->prof_ms = 0.0;
    h->prof_bytes = 0.0;
    return SA_OK;
  });
}

sa_status sa_profile_read(const sa_hierarchy *h, int64_t *launches, double *ms, double *bytes) {
  if (!h) return SA_ERR_INVALID_ARG;
  if (launches) *launches = h->prof_launches;
  if (ms) *ms = h->prof_ms;
  if (bytes) *bytes = h->prof_bytes;
  return SA_OK;
}

void sa_destroy(sa_hierarchy *h) {
  if (!h) return;
  try {
    (void)hipStreamSynchronize(h->stream);
    h->ar.release();
    (void)hipStreamSynchronize(h->stream);
  } catch (...) {
  }
  delete h;
}

const char *sa_status_string(sa_status s) {
  switch (s) {
    case SA_OK: return "ok";
    case SA_NOT_CONVERGED: return "not converged";
    case SA_PENDING: return "pending";
    case SA_ERR_INVALID_ARG: return "invalid argument";
    case SA_ERR_BAD_CSR: return "malformed CSR matrix";
    case SA_ERR_NONPOSITIVE_DIAG: return "zero or non-positive diagonal";
    case SA_ERR_NEGATIVE_EIGENVALUE: return "non-positive eigenvalue estimate";
    case SA_ERR_COARSEN_STALLED: return "coarsening stalled";
    case SA_ERR_COARSE_FACTOR: return "coarse factorisation failed";
    case SA_ERR_OOM: return "out of device memory";
    case SA_ERR_HIP: return "HIP runtime error";
    case SA_ERR_BREAKDOWN: return "CG breakdown";
  }
  return "unknown status";
}

const char *sa_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
