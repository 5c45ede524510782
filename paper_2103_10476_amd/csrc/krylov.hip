// GMRES building blocks (restarted flexible GMRES, Sec. 3.4): multi-vector canonical inner
// products, Gram-Schmidt updates, the Hessenberg column, Givens rotations and the
// least-squares back substitution.  Scalar steps run in one thread on the device, in the
// order of the textbook algorithm, so the iterates match a sequential implementation bit for
// bit.
#include "solve_device.hpp"

namespace sa {

// ---- GMRES building blocks ----------------------------------------------------------------
// Multi-vector canonical dot: the same blocks and trees as dot_f64, one per vector (grid.y).
__global__ __launch_bounds__(kBlock) void k_mdot_stage(const double *__restrict__ x,
                                                       int64_t ldx,
                                                       const double *__restrict__ y, int64_t m,
                                                       double *__restrict__ part,
                                                       int64_t ldp) {
  __shared__ double sh[kBlock];
  const int64_t v = blockIdx.y;
  dot_block(blockIdx.x, x + v * ldx, y, m, part + v * ldp + blockIdx.x, sh);
}
void multi_dot_f64(const double *V, int64_t ldv, int32_t nv, const double *w, int64_t n,
                   double *c, double *ws, hipStream_t s) {
  if (nv <= 0) return;
  int64_t m = n;
  const double *in = V;
  int64_t ldin = ldv;
  const double *iny = w;
  double *out = ws;
  for (;;) {
    int64_t nb = ceil_div(m, 4096);
    if (nb < 1) nb = 1;
    double *dst = (nb == 1) ? c : out;
    const int64_t ldo = (nb == 1) ? 1 : nb;
    k_mdot_stage<<<dim3((unsigned)nb, (unsigned)nv), kBlock, 0, s>>>(in, ldin, iny, m, dst, ldo);
    SA_LAUNCH_CHECK();
    if (nb == 1) break;
    in = out;
    ldin = nb;
    iny = nullptr;
    out += nb * nv;
    m = nb;
  }
}
__global__ void k_multi_axpy(const double *__restrict__ V, int64_t ldv, int32_t nv,
                             const double *__restrict__ c, double *__restrict__ w, int64_t n,
                             bool add) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double t = w[k];
  if (add)
    for (int32_t i = 0; i < nv; ++i) t = t + c[i] * V[i * ldv + k];
  else
    for (int32_t i = 0; i < nv; ++i) t = t - c[i] * V[i * ldv + k];
  w[k] = t;
}
void multi_axpy_f64(const double *V, int64_t ldv, int32_t nv, const double *c, double *w,
                    int64_t n, bool add, hipStream_t s) {
  if (n <= 0 || nv <= 0) return;
  k_multi_axpy<<<grid_for(n), kBlock, 0, s>>>(V, ldv, nv, c, w, n, add);
  SA_LAUNCH_CHECK();
}
__global__ void k_gmres_accum(double *H, int32_t m, int32_t j, const double *c, int32_t pass) {
  const int32_t i = threadIdx.x;
  if (i > j) return;
  H[(int64_t)i * m + j] = pass == 0 ? c[i] : H[(int64_t)i * m + j] + c[i];
}
void gmres_accum(double *H, int32_t m, int32_t j, const double *c, int32_t pass, hipStream_t s) {
  k_gmres_accum<<<1, (unsigned)ceil_div(j + 1, 64) * 64, 0, s>>>(H, m, j, c, pass);
  SA_LAUNCH_CHECK();
}
__global__ void k_gmres_norm(GmresScalars *S, double *H, int32_t m, int32_t j) {
  const double hn = sqrt(S->hn2);
  S->hn = hn;
  H[(int64_t)(j + 1) * m + j] = hn;
}
__global__ void k_div_scalar(const double *w, double *v, int64_t n, const double *den) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double d = *den;
  if (k < n && d > 0.0) v[k] = w[k] / d;
}
void gmres_normalize(GmresScalars *S, double *H, int32_t m, int32_t j, const double *w,
                     double *v, int64_t n, hipStream_t s) {
  k_gmres_norm<<<1, 1, 0, s>>>(S, H, m, j);
  k_div_scalar<<<grid_for(n), kBlock, 0, s>>>(w, v, n, &S->hn);
  SA_LAUNCH_CHECK();
}
__global__ void k_gmres_givens(double *H, int32_t m, int32_t j, double *cs, double *sn,
                               double *g, GmresScalars *S) {
  auto h = [&](int32_t i, int32_t k) -> double & { return H[(int64_t)i * m + k]; };
  for (int32_t i = 0; i < j; ++i) {
    const double t = cs[i] * h(i, j) + sn[i] * h(i + 1, j);
    h(i + 1, j) = -sn[i] * h(i, j) + cs[i] * h(i + 1, j);
    h(i, j) = t;
  }
  const double a = h(j, j), b = h(j + 1, j);
  if (b == 0.0) {
    cs[j] = 1.0;
    sn[j] = 0.0;
  } else {
    const double rho = sqrt(a * a + b * b);
    cs[j] = a / rho;
    sn[j] = b / rho;
  }
  h(j, j) = cs[j] * a + sn[j] * b;
  h(j + 1, j) = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  S->res = fabs(g[j + 1]);
}
void gmres_givens(double *H, int32_t m, int32_t j, double *cs, double *sn, double *g,
                  GmresScalars *S, hipStream_t s) {
  k_gmres_givens<<<1, 1, 0, s>>>(H, m, j, cs, sn, g, S);
  SA_LAUNCH_CHECK();
}
__global__ void k_gmres_backsolve(const double *H, int32_t m, int32_t k, const double *g,
                                  double *y, GmresScalars *S) {
  for (int32_t i = k - 1; i >= 0; --i) {
    double t = g[i];
    for (int32_t q = i + 1; q < k; ++q) t = t - H[(int64_t)i * m + q] * y[q];
    const double d = H[(int64_t)i * m + i];
    if (d == 0.0) S->err = 1;
    y[i] = t / d;
  }
}
void gmres_backsolve(const double *H, int32_t m, int32_t k, const double *g, double *y,
                     GmresScalars *S, hipStream_t s) {
  k_gmres_backsolve<<<1, 1, 0, s>>>(H, m, k, g, y, S);
  SA_LAUNCH_CHECK();
}
// (every entry of H and g that a cycle reads is written by that cycle first)
__global__ void k_gmres_beta(GmresScalars *S, double *g) {
  const double beta = sqrt(S->nrm2);
  S->beta = beta;
  g[0] = beta;
}
void gmres_start(GmresScalars *S, const double *r, double *v, int64_t n, double *g,
                 hipStream_t s) {
  k_gmres_beta<<<1, 1, 0, s>>>(S, g);
  k_div_scalar<<<grid_for(n), kBlock, 0, s>>>(r, v, n, &S->beta);
  SA_LAUNCH_CHECK();
}

}  // namespace sa
