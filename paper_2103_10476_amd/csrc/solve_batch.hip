// Grouped solve: CG + V-cycle for many hierarchies in lockstep.
//
// Each CG iteration of every running system is one "tick".  A tick's steps are the ones
// sa_solve takes for one system (preconditioner, inner products, scalar updates, fine-level
// SpMV), but each step is a single grouped launch over a table of segments, one segment per
// system, instead of one launch per system.  The kernels below look up their segment from
// the workgroup index and call the same device functions as the standalone kernels with the
// segment's own arguments (solve_device.hpp), and every system keeps its own vectors,
// scalars and reduction workspaces, so each system's arithmetic, iteration count and
// result are exactly those of sa_solve on it alone.
//
// Per tick the host records the launches and their segment tables into one descriptor
// buffer, copies it to the device once, launches, and reads back every system's CG scalars
// with one copy; systems that converged, failed or hit the iteration cap leave the group,
// new ones can join before any tick.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "batch.hpp"
#include "solve_device.hpp"

namespace sa {

// Segment of grid block g: the largest s with boff[s] <= g (boff ascending, boff[0] = 0).
__device__ __forceinline__ int32_t find_seg(const int32_t *boff, int32_t nseg, int32_t g) {
  int32_t lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (boff[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T, class Epi>
struct GSpmv {
  const int32_t *bstart, *rp, *col;
  const T *val, *x;
  Epi epi;
};

template <class T, class Epi>
__global__ __launch_bounds__(kBlock) void k_gspmv(const GSpmv<T, Epi> *segs,
                                                  const int32_t *boff, int32_t nseg) {
  __shared__ SpmvShared<T> sh;
  const int32_t g = xcd_block(blockIdx.x, gridDim.x);
  const int32_t s = find_seg(boff, nseg, g);
  const GSpmv<T, Epi> a = segs[s];
  spmv_block<T, Epi>(g - boff[s], a.bstart, a.rp, a.col, a.val, a.x, a.epi, sh);
}

enum GVecOp : int32_t {
  G_CHEB_FIRST_D, G_CHEB_FIRST_F, G_VEC_ADD_D, G_VEC_ADD_F, G_JAC_FIRST_D, G_JAC_FIRST_F,
  G_COPY_D, G_COPY_F, G_CAST_DF, G_CAST_FD, G_UPDATE_XR, G_UPDATE_P, G_VEC_SUB
};

struct GVec {
  int32_t op, n;
  const void *a, *b;
  void *c, *d;
  const PcgScalars *S;
  double sc;
  int32_t flag, pad;
};

__global__ __launch_bounds__(kBlock) void k_gvec(const GVec *segs, const int32_t *boff,
                                                 int32_t nseg) {
  const int32_t s = find_seg(boff, nseg, blockIdx.x);
  const GVec v = segs[s];
  const int32_t i = (blockIdx.x - boff[s]) * kBlock + threadIdx.x;
  if (i >= v.n) return;
  switch (v.op) {
    case G_CHEB_FIRST_D:
      cheb_first_at<double>(i, (const double *)v.a, (const double *)v.b, v.sc, (double *)v.c,
                            (double *)v.d, v.flag != 0);
      break;
    case G_CHEB_FIRST_F:
      cheb_first_at<float>(i, (const float *)v.a, (const float *)v.b, (float)v.sc,
                           (float *)v.c, (float *)v.d, v.flag != 0);
      break;
    case G_VEC_ADD_D: vec_add_at<double>(i, (double *)v.c, (const double *)v.a); break;
    case G_VEC_ADD_F: vec_add_at<float>(i, (float *)v.c, (const float *)v.a); break;
    case G_JAC_FIRST_D:
      jacobi_first_at<double>(i, (const double *)v.a, (const double *)v.b, v.sc,
                              (double *)v.c);
      break;
    case G_JAC_FIRST_F:
      jacobi_first_at<float>(i, (const float *)v.a, (const float *)v.b, (float)v.sc,
                             (float *)v.c);
      break;
    case G_COPY_D: ((double *)v.c)[i] = ((const double *)v.a)[i]; break;
    case G_COPY_F: ((float *)v.c)[i] = ((const float *)v.a)[i]; break;
    case G_CAST_DF: ((float *)v.c)[i] = (float)((const double *)v.a)[i]; break;
    case G_CAST_FD: ((double *)v.c)[i] = (double)((const float *)v.a)[i]; break;
    case G_UPDATE_XR:
      update_xr_at(i, (double *)v.c, (double *)v.d, (const double *)v.a, (const double *)v.b,
                   v.S->alpha);
      break;
    case G_UPDATE_P: update_p_at(i, (double *)v.c, (const double *)v.a, v.S->beta); break;
    case G_VEC_SUB:
      vec_sub_at(i, (const double *)v.a, (const double *)v.b, (double *)v.c);
      break;
    default: break;
  }
}

struct GGemv {
  int32_t n, pad;
  const double *M, *x;
  double *y;
};
__global__ __launch_bounds__(kBlock) void k_ggemv(const GGemv *segs, const int32_t *boff,
                                                  int32_t nseg) {
  const int32_t s = find_seg(boff, nseg, blockIdx.x);
  const GGemv a = segs[s];
  const int64_t row = (int64_t)(blockIdx.x - boff[s]) * (kBlock / 64) + (threadIdx.x >> 6);
  if (row < a.n) gemv_row(row, a.n, a.M, a.x, a.y);
}

struct GDot {
  const double *x, *y;
  int64_t n;
  double *out;  // block k writes out[k]
};
__global__ __launch_bounds__(kBlock) void k_gdot(const GDot *segs, const int32_t *boff,
                                                 int32_t nseg) {
  __shared__ double sh[kBlock];
  const int32_t s = find_seg(boff, nseg, blockIdx.x);
  const GDot a = segs[s];
  const int64_t blk = blockIdx.x - boff[s];
  dot_block(blk, a.x, a.y, a.n, a.out + blk, sh);
}

enum GScalOp : int32_t { G_ALPHA, G_BETA, G_INIT };
struct GScal {
  PcgScalars *S;
  int32_t op, pr;
};
__global__ void k_gscal(const GScal *segs, int32_t nseg) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const GScal a = segs[s];
  if (a.op == G_ALPHA) pcg_alpha_on(a.S);
  else if (a.op == G_BETA) pcg_beta_on(a.S, a.pr != 0);
  else pcg_init_on(a.S);
}

__global__ void k_ggather(PcgScalars *const *src, PcgScalars *dst, int32_t nseg) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) dst[s] = *src[s];
}

// ---- host side: recording a tick ------------------------------------------------------------
namespace {

// A recorded launch: the kernel (through a small trampoline), its segment table and block
// offsets (byte offsets into the descriptor buffer), the segment count and total blocks.
struct Rec {
  void (*launch)(const void *segs, const int32_t *boff, int32_t nseg, int32_t blocks,
                 hipStream_t s);
  size_t segs_off, boff_off;
  int32_t nseg, blocks;
};

template <class T, class Epi>
void launch_gspmv(const void *segs, const int32_t *boff, int32_t nseg, int32_t blocks,
                  hipStream_t s) {
  k_gspmv<T, Epi><<<(unsigned)blocks, kBlock, 0, s>>>((const GSpmv<T, Epi> *)segs, boff, nseg);
}
void launch_gvec(const void *segs, const int32_t *boff, int32_t nseg, int32_t blocks,
                 hipStream_t s) {
  k_gvec<<<(unsigned)blocks, kBlock, 0, s>>>((const GVec *)segs, boff, nseg);
}
void launch_ggemv(const void *segs, const int32_t *boff, int32_t nseg, int32_t blocks,
                  hipStream_t s) {
  k_ggemv<<<(unsigned)blocks, kBlock, 0, s>>>((const GGemv *)segs, boff, nseg);
}
void launch_gdot(const void *segs, const int32_t *boff, int32_t nseg, int32_t blocks,
                 hipStream_t s) {
  k_gdot<<<(unsigned)blocks, kBlock, 0, s>>>((const GDot *)segs, boff, nseg);
}
void launch_gscal(const void *segs, const int32_t *, int32_t nseg, int32_t, hipStream_t s) {
  k_gscal<<<grid_for(nseg), kBlock, 0, s>>>((const GScal *)segs, nseg);
}

// Builds the descriptor buffer of one tick.
struct Recorder {
  std::vector<uint8_t> buf;
  std::vector<Rec> recs;

  size_t put(const void *p, size_t bytes) {
    size_t off = (buf.size() + 15) & ~size_t(15);
    buf.resize(off + bytes);
    std::memcpy(buf.data() + off, p, bytes);
    return off;
  }
  // blocks[k] = blocks of segment k; empty segments are dropped by the callers
  template <class Seg>
  void add(void (*fn)(const void *, const int32_t *, int32_t, int32_t, hipStream_t),
           const std::vector<Seg> &segs, const std::vector<int32_t> &blocks) {
    if (segs.empty()) return;
    std::vector<int32_t> boff(segs.size() + 1, 0);
    for (size_t k = 0; k < segs.size(); ++k) boff[k + 1] = boff[k] + blocks[k];
    if (boff.back() == 0) return;
    Rec r;
    r.launch = fn;
    r.segs_off = put(segs.data(), sizeof(Seg) * segs.size());
    r.boff_off = put(boff.data(), sizeof(int32_t) * boff.size());
    r.nseg = (int32_t)segs.size();
    r.blocks = boff.back();
    recs.push_back(r);
  }
};

// The level data a V-cycle step touches, in the hierarchy's V-cycle precision.
template <class T>
struct View {
  const Csr *A, *P, *R;
  const T *Aval, *Pval, *Rval, *invD;
  T *f, *u, *r, *d1, *d2;
};
View<double> view_of(Level &L, double) {
  return {&L.A, &L.P, &L.R, L.A.val, L.P.val, L.R.val, L.sm_invD, L.f, L.u, L.r, L.d1, L.d2};
}
View<float> view_of(Level &L, float) {
  return {&L.A, &L.P, &L.R, L.Af, L.Pf, L.Rf, L.sm_invDf, L.ff, L.uf, L.rf, L.d1f, L.d2f};
}

template <class T, class Epi>
GSpmv<T, Epi> gspmv(const Csr &M, const T *val, const T *x, const Epi &e) {
  return GSpmv<T, Epi>{M.bstart, M.rp, M.col, val, x, e};
}

// One grouped SpMV launch over `items` (matrix, values, x, epilogue).
template <class T, class Epi>
void rec_spmv(Recorder &rc, const std::vector<GSpmv<T, Epi>> &segs,
              const std::vector<int32_t> &nblk) {
  std::vector<GSpmv<T, Epi>> s2;
  std::vector<int32_t> b2;
  for (size_t k = 0; k < segs.size(); ++k)
    if (nblk[k] > 0) {
      s2.push_back(segs[k]);
      b2.push_back(nblk[k]);
    }
  rc.add(launch_gspmv<T, Epi>, s2, b2);
}

void rec_vec(Recorder &rc, const std::vector<GVec> &segs) {
  std::vector<GVec> s2;
  std::vector<int32_t> b2;
  for (const GVec &v : segs)
    if (v.n > 0) {
      s2.push_back(v);
      b2.push_back((int32_t)grid_for(v.n));
    }
  rc.add(launch_gvec, s2, b2);
}

GVec gv(int32_t op, int32_t n, const void *a, const void *b, void *c, void *d = nullptr,
        double sc = 0.0, int32_t flag = 0, const PcgScalars *S = nullptr) {
  GVec v;
  v.op = op;
  v.n = n;
  v.a = a;
  v.b = b;
  v.c = c;
  v.d = d;
  v.S = S;
  v.sc = sc;
  v.flag = flag;
  v.pad = 0;
  return v;
}

// Canonical inner products res_k = x_k . y_k, one per system, with the stage structure of
// dot_f64: the first stage multiplies, later stages sum the previous stage's partials in the
// system's workspace, the last stage writes res_k.
struct DotJob {
  const double *x, *y;
  int64_t n;
  double *res, *ws;
};
void rec_dots(Recorder &rc, const std::vector<DotJob> &jobs) {
  struct St {
    const double *in, *iny;
    int64_t m;
    double *out;
    bool done;
  };
  std::vector<St> st;
  for (const DotJob &j : jobs) st.push_back({j.x, j.y, j.n, j.ws, false});
  for (;;) {
    std::vector<GDot> segs;
    std::vector<int32_t> blocks;
    bool any = false;
    for (size_t k = 0; k < st.size(); ++k) {
      St &a = st[k];
      if (a.done) continue;
      int64_t nb = ceil_div(a.m, 4096);
      if (nb < 1) nb = 1;
      double *dst = (nb == 1) ? jobs[k].res : a.out;
      segs.push_back({a.in, a.iny, a.m, dst});
      blocks.push_back((int32_t)nb);
      any = true;
      if (nb == 1) {
        a.done = true;
      } else {
        a.in = a.out;
        a.iny = nullptr;
        a.out += nb;
        a.m = nb;
      }
    }
    if (!any) break;
    rc.add(launch_gdot, segs, blocks);
  }
}

void rec_scal(Recorder &rc, const std::vector<GScal> &segs) {
  rc.add(launch_gscal, segs, std::vector<int32_t>(segs.size(), 1));
}

// ---- the grouped V-cycle (mirrors smooth / vcycle / coarse_apply of the standalone solve) --
struct Item {
  sa_hierarchy *h;
  int level;
  const void *f;  // T*
  void *u;        // T*
};

template <class T>
void rec_smooth(Recorder &rc, const std::vector<Item> &its, bool uzero) {
  if (its.empty()) return;
  const sa_options &o = its[0].h->opt;  // all items share smoother and degree
  std::vector<View<T>> v;
  for (const Item &it : its) v.push_back(view_of(it.h->lv[it.level], T()));
  const bool f32 = sizeof(T) == 4;
  if (o.smoother == SA_JACOBI) {
    int sweep = 0;
    if (uzero) {
      std::vector<GVec> g;
      for (size_t k = 0; k < its.size(); ++k) {
        const Level &L = its[k].h->lv[its[k].level];
        g.push_back(gv(f32 ? G_JAC_FIRST_F : G_JAC_FIRST_D, L.A.n, its[k].f, v[k].invD,
                       its[k].u, nullptr, (double)(T)L.jac_w));
      }
      rec_vec(rc, g);
      sweep = 1;
    }
    for (; sweep < o.degree; ++sweep) {
      std::vector<GSpmv<T, EpJacobi<T>>> sp;
      std::vector<int32_t> nb;
      std::vector<GVec> cp;
      for (size_t k = 0; k < its.size(); ++k) {
        const Level &L = its[k].h->lv[its[k].level];
        const T *u = (const T *)its[k].u;
        sp.push_back(gspmv<T>(*v[k].A, v[k].Aval, u,
                              EpJacobi<T>{u, (const T *)its[k].f, v[k].invD, (T)L.jac_w,
                                          v[k].d1}));
        nb.push_back(L.A.n > 0 ? L.A.nblk : 0);
        cp.push_back(gv(f32 ? G_COPY_F : G_COPY_D, L.A.n, v[k].d1, nullptr, its[k].u));
      }
      rec_spmv(rc, sp, nb);
      rec_vec(rc, cp);
    }
    return;
  }
  // Chebyshev
  std::vector<T *> dc, dn;
  std::vector<const T *> rin;
  for (size_t k = 0; k < its.size(); ++k) {
    dc.push_back(v[k].d1);
    dn.push_back(v[k].d2);
  }
  if (uzero) {
    std::vector<GVec> g;
    for (size_t k = 0; k < its.size(); ++k) {
      const Level &L = its[k].h->lv[its[k].level];
      g.push_back(gv(f32 ? G_CHEB_FIRST_F : G_CHEB_FIRST_D, L.A.n, its[k].f, v[k].invD, dc[k],
                     its[k].u, (double)(T)L.cheb_theta, o.degree == 1 ? 1 : 0));
      rin.push_back((const T *)its[k].f);
    }
    rec_vec(rc, g);
  } else {
    std::vector<GSpmv<T, EpChebStart<T>>> sp;
    std::vector<int32_t> nb;
    std::vector<GVec> add;
    for (size_t k = 0; k < its.size(); ++k) {
      const Level &L = its[k].h->lv[its[k].level];
      sp.push_back(gspmv<T>(*v[k].A, v[k].Aval, (const T *)its[k].u,
                            EpChebStart<T>{(const T *)its[k].f, v[k].invD, (T)L.cheb_theta,
                                           v[k].r, dc[k]}));
      nb.push_back(L.A.n > 0 ? L.A.nblk : 0);
      add.push_back(gv(f32 ? G_VEC_ADD_F : G_VEC_ADD_D, L.A.n, dc[k], nullptr, its[k].u));
      rin.push_back(v[k].r);
    }
    rec_spmv(rc, sp, nb);
    if (o.degree == 1) rec_vec(rc, add);
  }
  for (int m = 1; m < o.degree; ++m) {
    const bool last = (m == o.degree - 1);
    std::vector<GSpmv<T, EpChebStep<T>>> sp;
    std::vector<int32_t> nb;
    for (size_t k = 0; k < its.size(); ++k) {
      const Level &L = its[k].h->lv[its[k].level];
      sp.push_back(gspmv<T>(*v[k].A, v[k].Aval, dc[k],
                            EpChebStep<T>{dc[k], rin[k], v[k].invD, v[k].r, (T *)its[k].u,
                                          dn[k], (T)L.cheb_c1[m - 1], (T)L.cheb_c2[m - 1],
                                          uzero && m == 1, last}));
      nb.push_back(L.A.n > 0 ? L.A.nblk : 0);
      rin[k] = v[k].r;
      std::swap(dc[k], dn[k]);
    }
    rec_spmv(rc, sp, nb);
  }
}

template <class T>
void rec_coarse(Recorder &rc, const std::vector<Item> &its) {
  if (its.empty()) return;
  std::vector<GGemv> g;
  std::vector<int32_t> nb;
  if (sizeof(T) == 8) {
    for (const Item &it : its) {
      const Level &L = it.h->lv[it.level];
      g.push_back({L.A.n, 0, L.Ainv, (const double *)it.f, (double *)it.u});
      nb.push_back((int32_t)ceil_div(L.A.n, kBlock / 64));
    }
    rc.add(launch_ggemv, g, nb);
    return;
  }
  std::vector<GVec> c1, c2;
  for (const Item &it : its) {
    Level &L = it.h->lv[it.level];
    c1.push_back(gv(G_CAST_FD, L.A.n, it.f, nullptr, it.h->tmp64));
    g.push_back({L.A.n, 0, L.Ainv, it.h->tmp64, L.u});
    nb.push_back((int32_t)ceil_div(L.A.n, kBlock / 64));
    c2.push_back(gv(G_CAST_DF, L.A.n, L.u, nullptr, it.u));
  }
  rec_vec(rc, c1);
  rc.add(launch_ggemv, g, nb);
  rec_vec(rc, c2);
}

template <class T>
void rec_vcycle(Recorder &rc, const std::vector<Item> &its) {
  std::vector<Item> coarse, fine;
  for (const Item &it : its)
    (it.level + 1 == (int)it.h->lv.size() ? coarse : fine).push_back(it);
  rec_coarse<T>(rc, coarse);
  if (fine.empty()) return;
  rec_smooth<T>(rc, fine, true);
  std::vector<View<T>> v;
  for (const Item &it : fine) v.push_back(view_of(it.h->lv[it.level], T()));
  {
    std::vector<GSpmv<T, EpResid<T>>> sp;
    std::vector<int32_t> nb;
    for (size_t k = 0; k < fine.size(); ++k) {
      const Level &L = fine[k].h->lv[fine[k].level];
      sp.push_back(gspmv<T>(*v[k].A, v[k].Aval, (const T *)fine[k].u,
                            EpResid<T>{(const T *)fine[k].f, v[k].r}));
      nb.push_back(L.A.n > 0 ? L.A.nblk : 0);
    }
    rec_spmv(rc, sp, nb);
  }
  std::vector<Item> next;
  {
    std::vector<GSpmv<T, EpStore<T>>> sp;
    std::vector<int32_t> nb;
    for (size_t k = 0; k < fine.size(); ++k) {
      sa_hierarchy *h = fine[k].h;
      const Level &L = h->lv[fine[k].level];
      View<T> vc = view_of(h->lv[fine[k].level + 1], T());
      sp.push_back(gspmv<T>(L.R, v[k].Rval, v[k].r, EpStore<T>{vc.f}));
      nb.push_back(L.R.n > 0 ? L.R.nblk : 0);
      next.push_back({h, fine[k].level + 1, vc.f, vc.u});
    }
    rec_spmv(rc, sp, nb);
  }
  rec_vcycle<T>(rc, next);
  {
    std::vector<GSpmv<T, EpAdd<T>>> sp;
    std::vector<int32_t> nb;
    for (size_t k = 0; k < fine.size(); ++k) {
      const Level &L = fine[k].h->lv[fine[k].level];
      sp.push_back(gspmv<T>(L.P, v[k].Pval, (const T *)next[k].u, EpAdd<T>{(T *)fine[k].u}));
      nb.push_back(L.P.n > 0 ? L.P.nblk : 0);
    }
    rec_spmv(rc, sp, nb);
  }
  rec_smooth<T>(rc, fine, false);
}

// Systems whose V-cycles can share launches: same precision path, smoother and degree.
int64_t signature(const sa_hierarchy *h) {
  const bool f32 = h->opt.precision == SA_FP32_VCYCLE && h->lv.size() > 1;
  return ((int64_t)(f32 ? 1 : 0) << 40) | ((int64_t)h->opt.smoother << 32) | h->opt.degree;
}

// z = M^{-1} r for every system (precondition() of the standalone solve).
void rec_precondition(Recorder &rc, const std::vector<BatchSystem *> &sys) {
  std::vector<int64_t> sigs;
  for (BatchSystem *b : sys) {
    const int64_t sg = signature(b->h);
    if (std::find(sigs.begin(), sigs.end(), sg) == sigs.end()) sigs.push_back(sg);
  }
  for (int64_t sg : sigs) {
    std::vector<Item> d64, d32;
    std::vector<GVec> cin, cout;
    for (BatchSystem *b : sys) {
      sa_hierarchy *h = b->h;
      if (signature(h) != sg) continue;
      Level &L0 = h->lv[0];
      if (sg >> 40) {
        cin.push_back(gv(G_CAST_DF, h->n, h->r, nullptr, L0.ff));
        d32.push_back({h, 0, L0.ff, L0.uf});
        cout.push_back(gv(G_CAST_FD, h->n, L0.uf, nullptr, h->z));
      } else {
        d64.push_back({h, 0, h->r, h->z});
      }
    }
    if (!d32.empty()) {
      rec_vec(rc, cin);
      rec_vcycle<float>(rc, d32);
      rec_vec(rc, cout);
    }
    if (!d64.empty()) rec_vcycle<double>(rc, d64);
  }
}

}  // namespace

// ---- BatchSolver ---------------------------------------------------------------------------
BatchSolver::BatchSolver(hipStream_t s) : stream_(s) {}

BatchSolver::~BatchSolver() {
  if (dbuf_) dev_free(dbuf_, stream_);
  if (gbuf_) dev_free(gbuf_, stream_);
  if (hbuf_) (void)hipHostFree(hbuf_);
  if (hS_) (void)hipHostFree(hS_);
}

void BatchSolver::ensure(size_t desc_bytes, size_t nsys) {
  if (desc_bytes > dcap_) {
    if (dbuf_) dev_free(dbuf_, stream_);
    if (hbuf_) (void)hipHostFree(hbuf_);
    dbuf_ = nullptr;
    hbuf_ = nullptr;
    size_t c = 64 << 10;
    while (c < desc_bytes) c *= 2;
    dbuf_ = (uint8_t *)dev_alloc(c, stream_);
    SA_HIP(hipHostMalloc((void **)&hbuf_, c, hipHostMallocDefault));
    dcap_ = c;
  }
  if (nsys > gcap_) {
    if (gbuf_) dev_free(gbuf_, stream_);
    if (hS_) (void)hipHostFree(hS_);
    gbuf_ = nullptr;
    hS_ = nullptr;
    size_t c = 64;
    while (c < nsys) c *= 2;
    gbuf_ = (uint8_t *)dev_alloc(c * (sizeof(PcgScalars) + sizeof(void *)), stream_);
    SA_HIP(hipHostMalloc((void **)&hS_, c * sizeof(PcgScalars), hipHostMallocDefault));
    gcap_ = c;
  }
}

// Enqueues the recorded launches and a gather of the systems' scalars, then waits and
// copies the scalars to hS_.
void BatchSolver::run(void *recorder, const std::vector<BatchSystem *> &gather) {
  Recorder &rc = *(Recorder *)recorder;
  const size_t nsys = gather.size();
  std::vector<PcgScalars *> ptrs;
  for (BatchSystem *b : gather) ptrs.push_back(b->h->S);
  const size_t ptr_off = rc.put(ptrs.data(), sizeof(PcgScalars *) * nsys);
  ensure(rc.buf.size(), nsys);
  std::memcpy(hbuf_, rc.buf.data(), rc.buf.size());
  SA_HIP(hipMemcpyAsync(dbuf_, hbuf_, rc.buf.size(), hipMemcpyHostToDevice, stream_));
  for (const Rec &r : rc.recs) {
    r.launch(dbuf_ + r.segs_off, (const int32_t *)(dbuf_ + r.boff_off), r.nseg, r.blocks,
             stream_);
    SA_LAUNCH_CHECK();
  }
  if (nsys > 0) {
    PcgScalars *dst = (PcgScalars *)gbuf_;
    k_ggather<<<grid_for((int64_t)nsys), kBlock, 0, stream_>>>(
        (PcgScalars *const *)(dbuf_ + ptr_off), dst, (int32_t)nsys);
    SA_LAUNCH_CHECK();
    SA_HIP(hipMemcpyAsync(hS_, dst, sizeof(PcgScalars) * nsys, hipMemcpyDeviceToHost,
                          stream_));
  }
  SA_HIP(hipStreamSynchronize(stream_));
}

static void finish_copy(BatchSystem *b, hipStream_t s) {
  sa_hierarchy *h = b->h;
  if (!b->x || h->n <= 0) return;
  SA_HIP(hipMemcpyAsync(b->x, h->x, sizeof(double) * h->n,
                        b->loc == SA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        s));
}

// A system joins: r = b, x = 0, scalars cleared, r.r (the stopping test's reference).
void BatchSolver::add(BatchSystem *b) {
  sa_hierarchy *h = b->h;
  const sa_options &o = h->opt;
  b->pr = (o.pcg_beta == SA_BETA_PR) || (o.pcg_beta < 0 && o.precision == SA_FP32_VCYCLE);
  b->its = 0;
  b->phase = BatchSystem::kJoining;
  b->status = SA_NOT_CONVERGED;
  SA_HIP(hipMemcpyAsync(h->r, b->b, sizeof(double) * h->n,
                        b->loc == SA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        stream_));
  fill_f64(h->x, 0.0, h->n, stream_);
  fill_i32((int32_t *)h->S, 0, sizeof(PcgScalars) / sizeof(int32_t), stream_);
  joining_.push_back(b);
}

// One tick.  Joining systems get their reference r.r first (one readback for all of them);
// then every system runs the second half of its current CG iteration (preconditioner, r.z,
// beta, p) and, unless it reached the cap, the first half of the next (A p, alpha, x and r,
// r.r); one readback decides who continues.
void BatchSolver::tick(std::vector<BatchSystem *> &finished) {
  if (!joining_.empty()) {
    Recorder rc;
    std::vector<DotJob> dj;
    for (BatchSystem *b : joining_) dj.push_back({b->h->r, b->h->r, b->h->n, &b->h->S->rr, b->h->dws});
    rec_dots(rc, dj);
    run(&rc, joining_);
    for (size_t k = 0; k < joining_.size(); ++k) {
      BatchSystem *b = joining_[k];
      const double g0 = hS_[k].rr;
      b->g0 = g0;
      if (!std::isfinite(g0)) {
        b->status = SA_ERR_INVALID_ARG;
        b->phase = BatchSystem::kDone;
        finished.push_back(b);
        continue;
      }
      if (g0 == 0.0) {
        finish_copy(b, stream_);
        b->its = 0;
        b->relres = 0.0;
        b->status = SA_OK;
        b->phase = BatchSystem::kDone;
        finished.push_back(b);
        continue;
      }
      b->thr = (b->h->opt.rtol * b->h->opt.rtol) * g0;
      b->rr = g0;
      b->fresh = true;
      // with no iteration allowed only the preconditioner step runs (then the cap check)
      b->phase = b->h->opt.max_iter > 0 ? BatchSystem::kRunning : BatchSystem::kLastHalf;
      active_.push_back(b);
    }
    joining_.clear();
    SA_HIP(hipStreamSynchronize(stream_));
  }
  if (active_.empty()) return;
  Recorder rc;
  std::vector<BatchSystem *> cont_pr, all = active_, first;
  for (BatchSystem *b : active_) {
    if (!b->fresh && b->pr) cont_pr.push_back(b);
    if (b->phase != BatchSystem::kLastHalf) first.push_back(b);
  }
  // second half
  {
    std::vector<GVec> g;
    for (BatchSystem *b : cont_pr) g.push_back(gv(G_COPY_D, b->h->n, b->h->z, nullptr, b->h->zold));
    rec_vec(rc, g);
  }
  rec_precondition(rc, all);
  {
    std::vector<DotJob> dj;
    for (BatchSystem *b : all) dj.push_back({b->h->r, b->h->z, b->h->n, &b->h->S->rho1, b->h->dws});
    rec_dots(rc, dj);
  }
  if (!cont_pr.empty()) {
    std::vector<GVec> g;
    std::vector<DotJob> dj;
    for (BatchSystem *b : cont_pr) {
      g.push_back(gv(G_VEC_SUB, b->h->n, b->h->z, b->h->zold, b->h->w));
      dj.push_back({b->h->r, b->h->w, b->h->n, &b->h->S->rw, b->h->dws});
    }
    rec_vec(rc, g);
    rec_dots(rc, dj);
  }
  {
    std::vector<GScal> sc;
    std::vector<GVec> g;
    for (BatchSystem *b : all) {
      const bool fresh = b->fresh;
      sc.push_back({b->h->S, fresh ? G_INIT : G_BETA, b->pr ? 1 : 0});
      if (fresh) g.push_back(gv(G_COPY_D, b->h->n, b->h->z, nullptr, b->h->p));
      else g.push_back(gv(G_UPDATE_P, b->h->n, b->h->z, nullptr, b->h->p, nullptr, 0.0, 0, b->h->S));
    }
    rec_scal(rc, sc);
    rec_vec(rc, g);
  }
  // first half of the next iteration
  if (!first.empty()) {
    std::vector<GSpmv<double, EpStore<double>>> sp;
    std::vector<int32_t> nb;
    for (BatchSystem *b : first) {
      const Level &L0 = b->h->lv[0];
      sp.push_back(gspmv<double>(L0.A, L0.A.val, b->h->p, EpStore<double>{b->h->q}));
      nb.push_back(L0.A.n > 0 ? L0.A.nblk : 0);
    }
    rec_spmv(rc, sp, nb);
    std::vector<DotJob> dj;
    for (BatchSystem *b : first) dj.push_back({b->h->p, b->h->q, b->h->n, &b->h->S->pq, b->h->dws});
    rec_dots(rc, dj);
    std::vector<GScal> sc;
    for (BatchSystem *b : first) sc.push_back({b->h->S, G_ALPHA, 0});
    rec_scal(rc, sc);
    std::vector<GVec> g;
    for (BatchSystem *b : first)
      g.push_back(gv(G_UPDATE_XR, b->h->n, b->h->p, b->h->q, b->h->x, b->h->r, 0.0, 0, b->h->S));
    rec_vec(rc, g);
    dj.clear();
    for (BatchSystem *b : first) dj.push_back({b->h->r, b->h->r, b->h->n, &b->h->S->rr, b->h->dws});
    rec_dots(rc, dj);
  }
  run(&rc, all);
  std::vector<BatchSystem *> keep;
  for (size_t k = 0; k < all.size(); ++k) {
    BatchSystem *b = all[k];
    const PcgScalars &S = hS_[k];
    b->fresh = false;
    if (b->phase == BatchSystem::kLastHalf) {
      // the cap was reached; the final second half only feeds the breakdown check
      if (S.err) {
        b->status = SA_ERR_BREAKDOWN;
      } else {
        finish_copy(b, stream_);
        b->status = SA_NOT_CONVERGED;
        b->relres = std::sqrt(b->rr / b->g0);
      }
      b->phase = BatchSystem::kDone;
      finished.push_back(b);
      continue;
    }
    if (S.err) {
      b->status = SA_ERR_BREAKDOWN;
      b->phase = BatchSystem::kDone;
      finished.push_back(b);
      continue;
    }
    b->its += 1;
    b->rr = S.rr;
    if (b->rr <= b->thr) {
      finish_copy(b, stream_);
      b->status = SA_OK;
      b->relres = std::sqrt(b->rr / b->g0);
      b->phase = BatchSystem::kDone;
      finished.push_back(b);
      continue;
    }
    b->phase = (b->its >= b->h->opt.max_iter) ? BatchSystem::kLastHalf : BatchSystem::kRunning;
    keep.push_back(b);
  }
  active_.swap(keep);
  SA_HIP(hipStreamSynchronize(stream_));
}

extern thread_local std::string g_last_error;

}  // namespace sa

extern "C" sa_status sa_solve_many(sa_hierarchy *const *hs, int32_t count,
                                   const double *const *b, double *const *x, sa_location loc,
                                   int32_t *iterations, double *rel_residual,
                                   sa_status *status) {
  if (count < 0 || (count > 0 && (!hs || !b || !x || !status))) return SA_ERR_INVALID_ARG;
  if (count == 0) return SA_OK;
  for (int32_t k = 0; k < count; ++k)
    if (!hs[k] || !b[k] || !x[k] || !hs[k]->valid) return SA_ERR_INVALID_ARG;
  try {
    sa::BatchSolver bs(hs[0]->stream);
    std::vector<sa::BatchSystem> sys((size_t)count);
    for (int32_t k = 0; k < count; ++k) {
      sys[k].h = hs[k];
      sys[k].b = b[k];
      sys[k].x = x[k];
      sys[k].loc = loc;
      bs.add(&sys[k]);
    }
    std::vector<sa::BatchSystem *> fin;
    while (!bs.idle()) bs.tick(fin);
    for (int32_t k = 0; k < count; ++k) {
      status[k] = sys[k].status;
      if (iterations) iterations[k] = sys[k].its;
      if (rel_residual) rel_residual[k] = sys[k].relres;
    }
    return SA_OK;
  } catch (const sa::Error &e) {
    sa::g_last_error = e.what();
    return e.code;
  } catch (const std::exception &e) {
    sa::g_last_error = e.what();
    return SA_ERR_HIP;
  }
}
