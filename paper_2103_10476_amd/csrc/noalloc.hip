// sa_solve_gmres_noalloc: restarted GMRES on a set-up hierarchy that allocates no device
// memory, for callers that cannot allocate (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).  It runs the same iteration as sa_solve_gmres, whose
// workspace (Krylov basis, preconditioned vectors, Hessenberg matrix, rotations, inner-product
// partials, device scalars) comes from the library's memory cache for the call; here it lives
// in `scratch`, a fixed array of kScratchBytes compiled into the library, which each GPU the
// library runs on holds until the process ends.  Every call on a GPU shares that GPU's array,
// so calls that overlap on one GPU race; a call overwrites the whole workspace it uses
// before reading it, whatever an earlier call left there.
#include <mutex>
#include <string>

#include "hierarchy.hpp"

namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB
constexpr int kMaxDevices = 64;
}  // namespace

// In host code `scratch` names the symbol only: its address on a device comes from
// hipGetSymbolAddress (scratch_address), and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace sa {
extern thread_local std::string g_last_error;

namespace {
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];  // per device, looked up on the first call there

// Device address of `scratch` on the current device, looked up once per device.
void *scratch_address() {
  int dev = 0;
  SA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(SA_ERR_INVALID_ARG, "device ordinal >= 64");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    SA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(SA_ERR_HIP, "no device address for the scratch array");
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

// The fine-level SpMV timing creates HIP events on demand: off for the call.
struct ProfilingOff {
  sa_hierarchy *h;
  bool was;
  explicit ProfilingOff(sa_hierarchy *hh) : h(hh), was(hh->prof) { h->prof = false; }
  ~ProfilingOff() { h->prof = was; }
};
}  // namespace
}  // namespace sa

extern "C" sa_status sa_solve_gmres_noalloc(sa_hierarchy *h, const double *b, double *x,
                                            sa_location loc, int32_t restart,
                                            int32_t *iterations, double *rel_residual) {
  using namespace sa;
  if (!h || !b || !x) return SA_ERR_INVALID_ARG;
  try {
    if (restart < 1 || restart > 1024) throw Error(SA_ERR_INVALID_ARG, "restart not in 1..1024");
    const size_t need = gmres_work_bytes(h->n, restart);
    if (need > kScratchBytes)
      throw Error(SA_ERR_INVALID_ARG,
                  "GMRES workspace of " + std::to_string(need) + " bytes (n = " +
                      std::to_string(h->n) + ", restart = " + std::to_string(restart) +
                      ") exceeds the " + std::to_string(kScratchBytes) +
                      "-byte scratch array; use sa_solve_gmres or a smaller restart");
    void *base = scratch_address();
    ProfilingOff off(h);
    const sa_status st = gmres_run(h, b, x, loc, restart, gmres_work_carve(base, h->n, restart),
                                   true, iterations, rel_residual);
    if (st < 0) {
      (void)hipStreamSynchronize(h->stream);
      g_last_error = "GMRES breakdown (non-finite residual or singular least-squares system)";
    }
    return st;
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SA_ERR_OOM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return SA_ERR_HIP;
  }
}
