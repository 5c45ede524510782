// Grouped CG + V-cycle over many hierarchies (internal; solve_batch.hip).
#pragma once
#include <vector>

#include "hierarchy.hpp"

namespace sa {

// One system solved by a BatchSolver: A x = b on hierarchy h.  b and x stay owned by the
// caller and must remain valid until the system has finished.
struct BatchSystem {
  enum Phase { kJoining, kRunning, kLastHalf, kDone };
  sa_hierarchy *h = nullptr;
  const double *b = nullptr;
  double *x = nullptr;
  sa_location loc = SA_HOST;
  // results
  sa_status status = SA_NOT_CONVERGED;
  int32_t its = 0;
  double relres = 0.0;
  // state
  Phase phase = kJoining;
  bool pr = false, fresh = false;
  double g0 = 0.0, thr = 0.0, rr = 0.0;
  void *user = nullptr;
};

class BatchSolver {
 public:
  explicit BatchSolver(hipStream_t s);
  ~BatchSolver();
  BatchSolver(const BatchSolver &) = delete;
  BatchSolver &operator=(const BatchSolver &) = delete;
  // Queues a system; it joins the group at the next tick.
  void add(BatchSystem *b);
  // Advances every system by one CG iteration; systems that ended are appended to
  // `finished` (x written unless the status is an error).  Returns after the GPU is idle.
  void tick(std::vector<BatchSystem *> &finished);
  bool idle() const { return joining_.empty() && active_.empty(); }
  size_t active() const { return active_.size(); }

 private:
  void ensure(size_t desc_bytes, size_t nsys);
  void run(void *recorder, const std::vector<BatchSystem *> &gather);
  hipStream_t stream_;
  std::vector<BatchSystem *> joining_, active_;
  uint8_t *dbuf_ = nullptr, *hbuf_ = nullptr, *gbuf_ = nullptr;
  size_t dcap_ = 0, gcap_ = 0;
  PcgScalars *hS_ = nullptr;
};

}  // namespace sa
