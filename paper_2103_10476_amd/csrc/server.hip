// Serving runtime: many independent SA-AMG setup + solve requests on one GPU.
//
// Setup: each slot is a host worker thread with a HIP stream of its own.  Workers take
// requests in submission order while the admitted requests' device-byte estimates fit the
// budget, and run sa_setup on their slot's stream, so up to max_slots setups overlap on the
// GPU; a slot takes the next request as soon as its setup is done.
// Solve: one batcher thread owns every set-up request's solve.  Each tick advances all of
// them by one CG iteration with grouped launches (one kernel per V-cycle/CG step for all
// requests, solve_batch.hip); requests join at the next tick after their setup and leave when
// they converge, fail or hit the cap, and their device memory is released at once.
// Requests never share device memory (the caching allocator keeps blocks per stream, and
// each hierarchy keeps its own vectors and scalars), and the grouped kernels run each
// request's exact standalone arithmetic, so every result is independent of the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.hpp"

namespace sa {
extern thread_local std::string g_last_error;
}

namespace {

using sa::Error;

// Admission estimate (sa_estimate_bytes): bytes per stored entry of A, per row, and fixed.
constexpr int64_t kEstBytesPerEntry = 64;
constexpr int64_t kEstBytesPerRow = 1200;
constexpr int64_t kEstBytesFixed = 64ll << 20;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// A host copy of an input array, left uninitialised before the copy (no zero-fill pass).
template <class T>
struct HostCopy {
  std::unique_ptr<T[]> p;
  void reset() { p.reset(); }
};

struct Request {
  uint64_t ticket = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  // The inputs the setup and solve read: the request's own host copies (sa_server_submit) or
  // the caller's arrays (sa_server_submit_borrowed), in `loc` memory.
  const int32_t *rp = nullptr, *col = nullptr;
  const double *val = nullptr, *b = nullptr;
  sa_location loc = SA_HOST;
  HostCopy<int32_t> rp_copy, col_copy;
  HostCopy<double> val_copy, b_copy;
  sa_options opt{};
  std::vector<double> x;
  sa_result res{};
  std::string err;
  double t_submit = 0.0, t_solve = 0.0;
  bool done = false;
  sa::Meter meter;
  sa_hierarchy *h = nullptr;
  sa::BatchSystem sys;
};

}  // namespace

struct sa_server {
  std::mutex mu;
  std::condition_variable cv_work;   // workers: queue, budget or stop changed
  std::condition_variable cv_done;   // waiters: a request finished
  std::condition_variable cv_batch;  // batcher: a request is set up, or stop
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> ready;  // set up, waiting to join the solve group
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;  // not yet collected
  std::vector<std::thread> workers;
  std::thread batcher;
  std::vector<hipStream_t> streams;
  hipStream_t bstream = nullptr;
  int device = 0;
  int64_t budget = 0, reserved = 0, peak_reserved = 0;
  int64_t submitted = 0, completed = 0, failed = 0, running = 0;
  int64_t ticks = 0, tick_systems = 0, max_group = 0;
  uint64_t next_ticket = 1;
  bool stop = false, stop_batch = false;
  sa::Meter total;  // measured device bytes of all admitted requests
};

namespace {

void drop_inputs(Request &q) {
  q.rp_copy.reset();
  q.col_copy.reset();
  q.val_copy.reset();
  q.b_copy.reset();
  q.rp = q.col = nullptr;
  q.val = q.b = nullptr;
}

// Marks a request finished (its memory already released) and wakes waiters and workers.
void finalize(sa_server *s, Request &q) {
  int64_t peak = 0;
  sa::meter_read(&q.meter, nullptr, &peak);
  q.res.peak_bytes = peak;
  drop_inputs(q);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->reserved -= q.res.reserved_bytes;
    --s->running;
    if (q.res.status < 0) ++s->failed;
    else ++s->completed;
    q.res.latency_seconds = now_s() - q.t_submit;
    q.done = true;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// Setup on the slot's stream; a set-up request goes to the batcher.
void run_setup(sa_server *s, hipStream_t stream, const std::shared_ptr<Request> &qp) {
  Request &q = *qp;
  const double t_admit = now_s();
  q.res.queue_seconds = t_admit - q.t_submit;
  q.res.n = q.n;
  q.meter.parent = &s->total;
  sa::meter_begin(&q.meter);
  sa_context ctx{stream};
  sa_csr A{q.n, q.nnz, q.rp, q.col, q.val, q.loc};
  sa_hierarchy *h = nullptr;
  const sa_status st = sa_setup(&ctx, &A, nullptr, &q.opt, &h);
  sa::meter_end();
  q.t_solve = now_s();
  q.res.setup_seconds = q.t_solve - t_admit;
  if (st != SA_OK) {
    q.err = sa_last_error();
    q.res.status = st;
    finalize(s, q);
    return;
  }
  sa_info info;
  if (sa_hierarchy_info(h, &info) == SA_OK) q.res.levels = info.levels;
  q.rp_copy.reset();  // the matrix now lives in the hierarchy
  q.col_copy.reset();
  q.val_copy.reset();
  q.rp = q.col = nullptr;
  q.val = nullptr;
  q.h = h;
  q.x.assign((size_t)q.n, 0.0);
  q.sys.h = h;
  q.sys.b = q.b;
  q.sys.x = q.x.data();
  q.sys.loc = q.loc;
  q.sys.user = &q;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->ready.push_back(qp);
  }
  s->cv_batch.notify_all();
}

void worker_main(sa_server *s, int slot) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = s->streams[(size_t)slot];
  for (;;) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        if (s->stop) return true;
        if (s->queue.empty()) return false;
        const int64_t need = s->queue.front()->res.reserved_bytes;
        return s->running == 0 || s->reserved + need <= s->budget;
      });
      if (s->stop) return;
      q = s->queue.front();
      s->queue.pop_front();
      s->reserved += q->res.reserved_bytes;
      if (s->reserved > s->peak_reserved) s->peak_reserved = s->reserved;
      ++s->running;
    }
    run_setup(s, stream, q);
  }
}

const char *solve_message(sa_status st) {
  switch (st) {
    case SA_ERR_BREAKDOWN: return "CG breakdown (p'Ap <= 0 or r'z <= 0)";
    case SA_ERR_INVALID_ARG: return "non-finite right-hand side";
    default: return "solve failed";
  }
}

void batcher_main(sa_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_ptr<sa::BatchSolver> bs(new sa::BatchSolver(s->bstream));
  std::vector<std::shared_ptr<Request>> inflight;
  for (;;) {
    std::vector<std::shared_ptr<Request>> fresh;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_batch.wait(lk, [&] { return !s->ready.empty() || !bs->idle() || s->stop_batch; });
      if (s->ready.empty() && bs->idle()) return;  // stop_batch with nothing left
      fresh.swap(s->ready);
    }
    std::vector<sa::BatchSystem *> fin;
    try {
      for (auto &q : fresh) {
        bs->add(&q->sys);
        inflight.push_back(q);
      }
      bs->tick(fin);
    } catch (const std::exception &e) {
      // a runtime failure: every request in the group fails with it
      for (auto &q : inflight) {
        q->res.status = SA_ERR_HIP;
        q->err = e.what();
        (void)hipStreamSynchronize(s->bstream);
        sa::hierarchy_release_nosync(q->h);
        q->h = nullptr;
        finalize(s, *q);
      }
      inflight.clear();
      bs.reset(new sa::BatchSolver(s->bstream));
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      ++s->ticks;
      const int64_t g = (int64_t)(bs->active() + fin.size());
      s->tick_systems += g;
      s->max_group = std::max(s->max_group, g);
    }
    for (sa::BatchSystem *b : fin) {
      Request &q = *(Request *)b->user;
      q.res.status = b->status;
      q.res.iterations = b->its;
      q.res.rel_residual = b->relres;
      q.res.solve_seconds = now_s() - q.t_solve;
      if (b->status < 0) q.err = solve_message(b->status);
      sa::hierarchy_release_nosync(q.h);  // the batcher's stream is idle after a tick
      q.h = nullptr;
      finalize(s, q);
      inflight.erase(std::find_if(inflight.begin(), inflight.end(),
                                  [&](const std::shared_ptr<Request> &r) { return r.get() == &q; }));
    }
  }
}

template <class F>
sa_status guarded_server(F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    sa::g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    sa::g_last_error = "host allocation failed";
    return SA_ERR_OOM;
  } catch (const std::exception &e) {
    sa::g_last_error = e.what();
    return SA_ERR_HIP;
  }
}

template <class T>
const T *copy_host(HostCopy<T> &dst, const T *src, size_t count, sa_location loc) {
  if (count == 0) return nullptr;
  if (!src) throw Error(SA_ERR_INVALID_ARG, "null array");
  dst.p.reset(new T[count]);
  if (loc == SA_DEVICE) {
    SA_HIP(hipMemcpy(dst.p.get(), src, sizeof(T) * count, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(dst.p.get(), src, sizeof(T) * count);
  }
  return dst.p.get();
}

// Writes a finished request's result and returns its status; the caller holds s->mu and
// removes the ticket afterwards.
sa_status collect(Request &q, double *x, sa_location loc, sa_result *r) {
  if (r) *r = q.res;
  if (q.res.status < 0) {
    sa::g_last_error = q.err;
    return (sa_status)q.res.status;
  }
  if (x && q.n > 0) {
    if (loc == SA_DEVICE) {
      SA_HIP(hipMemcpy(x, q.x.data(), sizeof(double) * (size_t)q.n, hipMemcpyHostToDevice));
    } else {
      std::memcpy(x, q.x.data(), sizeof(double) * (size_t)q.n);
    }
  }
  return (sa_status)q.res.status;
}

}  // namespace

extern "C" {

int64_t sa_estimate_bytes(int32_t n, int64_t nnz) {
  if (n < 0 || nnz < 0) return 0;
  // per stored entry of A and per row, with head-room for operator complexity ~3 and for
  // the Galerkin products' temporaries; plus a fixed allowance for small problems
  return (int64_t)kEstBytesPerEntry * nnz + (int64_t)kEstBytesPerRow * n + kEstBytesFixed;
}

sa_status sa_server_create(const sa_context *ctx, size_t hbm_budget, int32_t max_slots,
                           sa_server **out) {
  if (!out) return SA_ERR_INVALID_ARG;
  *out = nullptr;
  if (hbm_budget == 0 || max_slots < 1 || max_slots > 32) return SA_ERR_INVALID_ARG;
  (void)ctx;
  return guarded_server([&]() -> sa_status {
    std::unique_ptr<sa_server> s(new sa_server());
    SA_HIP(hipGetDevice(&s->device));
    s->budget = (int64_t)std::min<size_t>(hbm_budget, (size_t)INT64_MAX);
    for (int i = 0; i < max_slots; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        for (auto x : s->streams) (void)hipStreamDestroy(x);
        throw Error(SA_ERR_HIP, "hipStreamCreateWithFlags failed");
      }
      s->streams.push_back(st);
    }
    if (hipStreamCreateWithFlags(&s->bstream, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      throw Error(SA_ERR_HIP, "hipStreamCreateWithFlags failed");
    }
    for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker_main, s.get(), i);
    s->batcher = std::thread(batcher_main, s.get());
    *out = s.release();
    return SA_OK;
  });
}

}  // extern "C"

namespace {

// Common part of the two submission calls: checks, admission estimate, inputs (copied or
// borrowed), queueing.
sa_status submit_request(sa_server *s, const sa_csr *A, const double *b, const sa_options *o,
                         uint64_t *ticket, bool borrow) {
  if (!s || !A || !b || !ticket) return SA_ERR_INVALID_ARG;
  if (A->n <= 0 || A->nnz < 0 || A->nnz >= (int64_t)INT32_MAX || !A->row_ptr)
    return SA_ERR_INVALID_ARG;
  if (A->nnz > 0 && (!A->col || !A->val)) return SA_ERR_INVALID_ARG;
  if (A->loc != SA_HOST && A->loc != SA_DEVICE) return SA_ERR_INVALID_ARG;
  if (o && o->struct_size != sizeof(sa_options)) return SA_ERR_INVALID_ARG;
  return guarded_server([&]() -> sa_status {
    auto q = std::make_shared<Request>();
    q->n = A->n;
    q->nnz = A->nnz;
    if (o) q->opt = *o;
    else sa_default_options(&q->opt);
    q->res.reserved_bytes = sa_estimate_bytes(A->n, A->nnz);
    if (q->res.reserved_bytes > s->budget)
      throw Error(SA_ERR_OOM, "request estimate exceeds the server's memory budget");
    if (borrow) {
      q->rp = A->row_ptr;
      q->col = A->col;
      q->val = A->val;
      q->b = b;
      q->loc = A->loc;
    } else {
      q->rp = copy_host(q->rp_copy, A->row_ptr, (size_t)A->n + 1, A->loc);
      q->col = copy_host(q->col_copy, A->col, (size_t)A->nnz, A->loc);
      q->val = copy_host(q->val_copy, A->val, (size_t)A->nnz, A->loc);
      q->b = copy_host(q->b_copy, b, (size_t)A->n, A->loc);
      q->loc = SA_HOST;
    }
    q->t_submit = now_s();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) throw Error(SA_ERR_INVALID_ARG, "server is shutting down");
      q->ticket = s->next_ticket++;
      s->all[q->ticket] = q;
      s->queue.push_back(q);
      ++s->submitted;
      *ticket = q->ticket;
    }
    s->cv_work.notify_all();
    return SA_OK;
  });
}

}  // namespace

extern "C" {

sa_status sa_server_submit(sa_server *s, const sa_csr *A, const double *b, const sa_options *o,
                           uint64_t *ticket) {
  return submit_request(s, A, b, o, ticket, false);
}

sa_status sa_server_submit_borrowed(sa_server *s, const sa_csr *A, const double *b,
                                    const sa_options *o, uint64_t *ticket) {
  return submit_request(s, A, b, o, ticket, true);
}

sa_status sa_server_poll(sa_server *s, uint64_t ticket, double *x, sa_location loc,
                         sa_result *r) {
  if (!s) return SA_ERR_INVALID_ARG;
  return guarded_server([&]() -> sa_status {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) throw Error(SA_ERR_INVALID_ARG, "unknown ticket");
    if (!it->second->done) return SA_PENDING;
    std::shared_ptr<Request> q = it->second;
    s->all.erase(it);
    return collect(*q, x, loc, r);
  });
}

sa_status sa_server_wait(sa_server *s, uint64_t ticket, double *x, sa_location loc,
                         sa_result *r) {
  if (!s) return SA_ERR_INVALID_ARG;
  return guarded_server([&]() -> sa_status {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) throw Error(SA_ERR_INVALID_ARG, "unknown ticket");
    std::shared_ptr<Request> q = it->second;
    s->cv_done.wait(lk, [&] { return q->done; });
    s->all.erase(ticket);
    return collect(*q, x, loc, r);
  });
}

sa_status sa_server_drain(sa_server *s) {
  if (!s) return SA_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
  return SA_OK;
}

sa_status sa_server_get_stats(const sa_server *cs, sa_server_stats *st) {
  if (!cs || !st) return SA_ERR_INVALID_ARG;
  sa_server *s = const_cast<sa_server *>(cs);
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->queued = (int64_t)s->queue.size();
  st->running = s->running;
  st->budget_bytes = s->budget;
  st->reserved_bytes = s->reserved;
  st->peak_reserved_bytes = s->peak_reserved;
  sa::meter_read(&s->total, nullptr, &st->peak_measured_bytes);
  st->solve_ticks = s->ticks;
  st->mean_group = s->ticks ? (double)s->tick_systems / (double)s->ticks : 0.0;
  st->max_group = s->max_group;
  return SA_OK;
}

void sa_server_destroy(sa_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();  // setups in progress finish and go to the batcher
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop_batch = true;
  }
  s->cv_batch.notify_all();
  if (s->batcher.joinable()) s->batcher.join();  // solves in progress finish
  for (auto st : s->streams) {
    sa::dev_release_stream(st);
    (void)hipStreamDestroy(st);
  }
  if (s->bstream) {
    sa::dev_release_stream(s->bstream);
    (void)hipStreamDestroy(s->bstream);
  }
  delete s;
}

}  // extern "C"
