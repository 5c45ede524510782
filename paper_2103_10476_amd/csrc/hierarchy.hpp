// Internal layout of a hierarchy (shared by the host runtime and the grouped solver).
#pragma once
#include <vector>

#include "kernels.hpp"

namespace sa {

constexpr int32_t kMaxDense = 8192;

struct Level {
  Csr A;                  // operator of this level
  Csr As;                 // matrix the prolongator is built from (A, or D_B A D_B on level 0)
  uint8_t *mask = nullptr;
  int32_t *agg = nullptr;
  uint8_t *is_root = nullptr;
  int32_t nc = 0;
  int32_t mis_rounds = 0;
  bool wave_rows = false;  // rows long enough for the wavefront-per-row setup kernels
  double *xyz = nullptr;   // node coordinates (n x dim) when the distance strength is used
  // systems SA: dofs per node, node graph and labels, QR tentative prolongator, this level's
  // nullspace (n x k) and the next level's (nc k x k)
  int32_t bs = 1;
  Csr Gn;
  uint8_t *nmask = nullptr;
  Csr Pt;
  double *B = nullptr, *Bc = nullptr;
  Csr Abar;
  double *invD = nullptr;
  double *lam_d = nullptr, *omega_d = nullptr;
  double lam = 0.0, omega = 0.0;
  Csr P, R;
  double *sm_invD = nullptr;
  double *sm_lam_d = nullptr;
  double sm_lam = 0.0;
  bool sm_pending = false;  // sm_invD / sm_lam_d queued on the side stream, not yet joined
  double cheb_theta = 0.0;
  std::vector<double> cheb_c1, cheb_c2;  // per Chebyshev step m = 1..deg-1
  double jac_w = 0.0;
  double *Ainv = nullptr;  // coarsest only: dense inverse, row-major
  Sell Aell;  // sliced-ELL copy of A for the solve (when it pays; see sell_build)
  // re-setup plans, built by the first numeric re-setup: A P kept with its pattern, the
  // numeric plans of A P and R (A P), and the positions of P's entries in R
  bool planned = false;
  Csr APk;
  SpgemmPlan pap, prap;
  int32_t *rperm = nullptr;
  // FP32 copies (FP32 V-cycle)
  float *Af = nullptr, *Pf = nullptr, *Rf = nullptr, *sm_invDf = nullptr;
  // work vectors
  double *f = nullptr, *u = nullptr, *r = nullptr, *d1 = nullptr, *d2 = nullptr;
  float *ff = nullptr, *uf = nullptr, *rf = nullptr, *d1f = nullptr, *d2f = nullptr;
};

}  // namespace sa

struct sa_hierarchy {
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;   // side stream used during the setup (see side_stream)
  sa_options opt{};
  sa::Arena ar;
  std::vector<sa::Level> lv;
  int32_t *err = nullptr;
  double setup_seconds = 0.0;
  bool valid = true;            // false after a failed re-setup
  int32_t dim = 0;              // > 0: distance-Laplacian strength from coordinates
  int32_t k = 0;                // > 0: systems SA with a k-vector nullspace
  double *dB = nullptr;         // nullspace vector (when it is not all ones)
  double *As0 = nullptr;        // D_B A D_B values on level 0 (when scaled)
  // solve workspace
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *zold = nullptr,
         *w = nullptr, *dws = nullptr, *tmp64 = nullptr;
  sa::PcgScalars *S = nullptr;
  int32_t n = 0;
  // fine-level SpMV timing (sa_profile_enable)
  bool prof = false;
  std::vector<hipEvent_t> ev;   // event pool, pairs (start, stop)
  std::vector<double> ev_bytes; // algorithmic bytes of each recorded pair
  int32_t nev = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0.0, prof_bytes = 0.0;
  ~sa_hierarchy() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

namespace sa {
void hierarchy_release_nosync(sa_hierarchy *h);

// Restarted flexible GMRES on a set-up hierarchy with a caller-provided workspace.
struct GmresWork {
  double *V, *Z, *H, *cs, *sn, *g, *y, *c, *ws;
  GmresScalars *S;
};
// Bytes of the workspace for n unknowns and restart m (parts 256-byte aligned), and its
// layout within a block of that size starting at a 256-byte boundary.
size_t gmres_work_bytes(int32_t n, int32_t m);
GmresWork gmres_work_carve(void *base, int32_t n, int32_t m);
// The GMRES iteration (see hierarchy.hip).  Throws sa::Error on invalid input.
sa_status gmres_run(sa_hierarchy *h, const double *b, double *x, sa_location loc,
                    int32_t restart, const GmresWork &wk, bool direct_reads,
                    int32_t *iterations, double *relres);
}  // namespace sa
