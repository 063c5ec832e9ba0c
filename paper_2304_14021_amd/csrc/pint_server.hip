// Serving loop: a persistent worker thread that admits all-at-once solves as
// HBM and streams free up, runs their outer iterations concurrently on
// separate HIP streams (one per active slot), captures each request's outer
// iteration once as a HIP graph and replays it for the iterations after the
// first, and retires each request as soon as its own stop flag is set.  Requests never wait for
// each other's iterations: continuous batching at iteration granularity.
//
// Memory: every request's device state (plan tables, u0, U, workspace) is a
// sub-allocation of the caller's pool (first-fit, coalescing free list).  A
// request is admitted only when its whole footprint fits, so the server never
// allocates device memory itself and never calls hipFree while work runs.
// Results of host-buffer requests go to a pinned host result pool allocated
// once at creation, where they wait for pint_server_wait.
//
// Threads: every HIP call of a server is made by its worker thread (besides
// creation and destruction).  Client threads only validate, queue, and copy
// finished results out of pinned host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "pint.h"
#include "pint_internal.hpp"

using namespace pint;

namespace {

using Clock = std::chrono::steady_clock;

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

enum ReqState { RQ_QUEUED, RQ_ACTIVE, RQ_DONE };

struct Req {
  uint64_t ticket = 0;
  pint_problem prob{};
  pint_plan* plan = nullptr;
  std::vector<double> u0;
  size_t h_off = 0;              // pinned result block (host-buffer requests)
  bool h_held = false;           // the block holds the finished U until wait
  const double* d_u0 = nullptr;  // caller-owned device input (device-resident requests)
  double* d_U = nullptr;         // caller-owned device state and result
  pint_report rep{};
  int status = PINT_OK;
  std::string err;  // message of a worker-side failure
  ReqState state = RQ_QUEUED;
  bool cancel = false;
  bool waited = false;  // a pint_server_wait call holds this ticket
  size_t ns = 0, nt = 0;
  size_t tab_bytes = 0, work_bytes = 0, footprint = 0;
  size_t pool_off = 0;
  Clock::time_point t_submit, t_admit, t_done;
};

enum SlotState { SL_IDLE, SL_RUNNING, SL_DRAINING };

// Everything that selects kernels or changes the iteration count of a
// request: dim, n, nt, precision, flags, operator, time path, theta.
using ShapeKey = std::tuple<int, int, int, int, unsigned, int, int, double>;

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  Ctrl* h_ctrl = nullptr;  // pinned status mirror of the running request
  double* h_in = nullptr;  // pinned staging for u0
  size_t in_cap = 0;
  SlotState state = SL_IDLE;
  Req* req = nullptr;
  int it_enq = 0;
  double* d_u0 = nullptr;
  double* d_U = nullptr;
  void* d_work = nullptr;
  hipGraphExec_t graph = nullptr;  // the running request's captured iteration
  ShapeKey cur_key{};
};

// First-fit allocator over [0, size) with coalescing.
class PoolAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  bool alloc(size_t len, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        const size_t rest = it->second - len, start = it->first + len;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += len;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t len) {
    used_ -= len;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

}  // namespace

struct pint_server {
  pint_server_config cfg{};
  int device = 0;
  unsigned char* pool = nullptr;
  PoolAlloc alloc;
  unsigned char* h_pool = nullptr;  // pinned host result pool
  PoolAlloc h_alloc;
  std::vector<Slot> slots;
  std::deque<Req*> queue;
  std::map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::thread worker;
  std::map<ShapeKey, int> predict;  // iterations the last request of a shape class needed
  // statistics
  uint64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_cancelled = 0;
  uint64_t graph_captures = 0, graph_updates = 0, graph_launches = 0;
  size_t pool_peak = 0;
  std::vector<double> lat_ms;
  double dof_done = 0.0;
  double host_seconds = 0.0;  // worker time spent admitting and advancing requests
  bool have_first = false;
  Clock::time_point t_first, t_last;
  int fatal = PINT_OK;     // PINT_EHIP after a HIP error: no further admissions
  std::string fatal_msg;   // what failed
};

namespace {

thread_local std::string g_srv_err;

// Record a HIP error that ends the server's service: later submissions fail
// and queued requests are finished with it.  Lock held.
void set_fatal(pint_server* s, const std::string& msg) {
  if (s->fatal == PINT_OK) {
    s->fatal = PINT_EHIP;
    s->fatal_msg = msg;
  }
}

// Errors are per calling thread; a request's worker-side error travels with
// the request and becomes the waiting thread's error.
int srv_fail(pint_server*, int code, const std::string& msg) {
  g_srv_err = msg;
  return code;
}

ShapeKey key_of(const pint_problem& p) {
  return ShapeKey(p.dim, p.nx, p.nt, p.precision, p.flags, p.op, p.time_path, p.theta);
}

// Destroy the slot's executable graph (its request has retired).
void drop_graph(Slot& sl) {
  if (sl.graph) (void)hipGraphExecDestroy(sl.graph);
  sl.graph = nullptr;
}

void finish_req(pint_server* s, Req* r, int status) {
  r->status = status;
  if (status != PINT_OK && status != PINT_ECANCELED && status != PINT_ENOCONV && status != PINT_EDIVERGED) {
    // the failing worker-side call left its message on the plan or here
    const char* pe = r->plan ? pint_plan_last_error(r->plan) : nullptr;
    r->err = (pe && *pe) ? std::string(pe) : g_srv_err;
  }
  r->state = RQ_DONE;
  r->t_done = Clock::now();
  if (r->plan) {
    pint_plan_destroy(r->plan);
    r->plan = nullptr;
  }
  if (status == PINT_ECANCELED) {
    ++s->n_cancelled;
  } else if (status == PINT_OK) {
    ++s->n_completed;
    s->lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
    s->dof_done += double(r->ns) * double(r->nt);
    s->t_last = r->t_done;
  } else {
    ++s->n_failed;
  }
  s->cv_done.notify_all();
}

// Enqueue iteration `it` of the slot's request: the first one directly (it
// reads the broadcast datum); later ones by replaying a graph of one outer
// iteration, captured for this request when its second iteration is
// enqueued.  A graph is never re-targeted to another request (no
// hipGraphExecUpdate): each request gets its own capture and instantiation,
// and the executable graph is destroyed when the request retires.  Called by
// the worker thread only.
int enqueue_it(pint_server* s, Slot& sl, int it) {
  Req* r = sl.req;
  if (it == 0 || (s->cfg.flags & PINT_SERVER_NO_GRAPHS)) {
    return solve_enqueue(r->plan, sl.d_u0, sl.d_U, sl.d_work, r->work_bytes, sl.st, sl.h_ctrl, it);
  }
  if (!sl.graph) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(sl.st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return srv_fail(s, PINT_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    const int rc = solve_enqueue(r->plan, sl.d_u0, sl.d_U, sl.d_work, r->work_bytes, sl.st, sl.h_ctrl, 1);
    e = hipStreamEndCapture(sl.st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return srv_fail(s, PINT_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      sl.graph = nullptr;
      return srv_fail(s, PINT_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    ++s->graph_captures;
  }
  const hipError_t e = hipGraphLaunch(sl.graph, sl.st);
  if (e != hipSuccess) return srv_fail(s, PINT_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  ++s->graph_launches;
  return PINT_OK;
}

bool grow_pinned(double** p, size_t* cap, size_t need) {
  if (*cap >= need) return true;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(p), need * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return false;
  *cap = need;
  return true;
}

// Admit request r into slot sl at pool offset off.  Lock held.
int start_req(pint_server* s, Slot& sl, Req* r) {
  unsigned char* base = s->pool + r->pool_off;
  void* d_tab = base;
  base += al256(r->tab_bytes);
  sl.d_u0 = reinterpret_cast<double*>(base);
  base += al256(r->ns * sizeof(double));
  sl.d_U = reinterpret_cast<double*>(base);
  base += al256(r->ns * r->nt * sizeof(double));
  sl.d_work = base;
  int rc = PINT_OK;
  if (r->d_U) {
    sl.d_work = sl.d_u0;  // no u0/U in the pool: the workspace follows the tables
    sl.d_u0 = const_cast<double*>(r->d_u0);
    sl.d_U = r->d_U;
    rc = plan_bind_tables(r->plan, d_tab, sl.st, true);
    if (rc) return rc;
  } else {
    if (!grow_pinned(&sl.h_in, &sl.in_cap, r->ns))
      return srv_fail(s, PINT_ENOMEM, "pinned staging allocation failed");
    rc = plan_bind_tables(r->plan, d_tab, sl.st, true);
    if (rc) return rc;
    std::memcpy(sl.h_in, r->u0.data(), r->ns * sizeof(double));
    if (hipMemcpyAsync(sl.d_u0, sl.h_in, r->ns * sizeof(double), hipMemcpyHostToDevice, sl.st) != hipSuccess)
      return srv_fail(s, PINT_EHIP, "u0 copy failed");
  }
  rc = solve_begin(r->plan, sl.d_u0, sl.d_U, sl.d_work, r->work_bytes, sl.st, sl.h_ctrl);
  if (rc) return rc;
  sl.req = r;
  sl.cur_key = key_of(r->prob);
  drop_graph(sl);
  sl.it_enq = 0;
  const int maxit = plan_max_iter(r->plan);
  auto pr = s->predict.find(sl.cur_key);
  const int first = std::min(maxit, std::max(2, pr == s->predict.end() ? 2 : pr->second));
  for (int it = 0; it < first; ++it) {
    rc = enqueue_it(s, sl, it);
    if (rc) return rc;
    ++sl.it_enq;
  }
  if (hipEventRecord(sl.ev, sl.st) != hipSuccess) return srv_fail(s, PINT_EHIP, "hipEventRecord failed");
  sl.state = SL_RUNNING;
  r->state = RQ_ACTIVE;
  r->t_admit = Clock::now();
  if (!s->have_first) {
    s->have_first = true;
    s->t_first = r->t_admit;
  }
  return PINT_OK;
}

// Advance a slot whose last event completed.  Running: retire the request
// if it has stopped (a host-buffer request first copies U into its pinned
// result block and drains), else enqueue one more iteration.  Draining: the
// copy is done; release the device block.  Lock held.
int advance(pint_server* s, Slot& sl) {
  Req* r = sl.req;
  if (sl.state == SL_RUNNING) {
    const Ctrl& c = *sl.h_ctrl;
    const bool done = reinterpret_cast<const volatile int&>(c.done) != 0;
    const int maxit = plan_max_iter(r->plan);
    if (!(r->cancel || done || sl.it_enq >= maxit)) {
      int rc = enqueue_it(s, sl, sl.it_enq);
      if (rc) return rc;
      ++sl.it_enq;
      if (hipEventRecord(sl.ev, sl.st) != hipSuccess) return srv_fail(s, PINT_EHIP, "hipEventRecord failed");
      return PINT_OK;
    }
    // every enqueued iteration has finished (the slot's event completed)
    r->status = r->cancel ? PINT_ECANCELED : solve_status(r->plan, c, &r->rep);
    if (r->status == PINT_OK) s->predict[sl.cur_key] = c.iter;
    sl.state = SL_DRAINING;
    if (!r->cancel && !r->d_U) {
      void* dst = s->h_pool + r->h_off;
      if (hipMemcpyAsync(dst, sl.d_U, r->ns * r->nt * sizeof(double), hipMemcpyDeviceToHost, sl.st) != hipSuccess)
        return srv_fail(s, PINT_EHIP, "result copy failed");
      if (hipEventRecord(sl.ev, sl.st) != hipSuccess) return srv_fail(s, PINT_EHIP, "hipEventRecord failed");
      r->h_held = true;
      return PINT_OK;
    }
  }
  // draining (or nothing to copy): release the device block and retire
  r->rep.struct_size = sizeof(pint_report);
  r->rep.ms_total = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
  s->alloc.release(r->pool_off, r->footprint);
  if (!r->h_held && !r->d_U) s->h_alloc.release(r->h_off, r->ns * r->nt * sizeof(double));
  drop_graph(sl);
  sl.req = nullptr;
  sl.state = SL_IDLE;
  finish_req(s, r, r->status);
  return PINT_OK;
}

void worker_main(pint_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    bool progressed = false;
    // after a HIP error nothing more is admitted: queued requests fail with it
    while (s->fatal != PINT_OK && !s->queue.empty()) {
      Req* r = s->queue.front();
      s->queue.pop_front();
      g_srv_err = "server stopped after a HIP error: " + s->fatal_msg;
      finish_req(s, r, PINT_EHIP);
      progressed = true;
    }
    // admission, first come first served, as slots and pool memory allow
    while (!s->queue.empty() && s->fatal == PINT_OK) {
      Req* r = s->queue.front();
      if (r->cancel) {
        s->queue.pop_front();
        finish_req(s, r, PINT_ECANCELED);
        progressed = true;
        continue;
      }
      Slot* free_slot = nullptr;
      for (auto& sl : s->slots)
        if (sl.state == SL_IDLE) {
          free_slot = &sl;
          break;
        }
      if (!free_slot) break;
      size_t off = 0, hoff = 0;
      const size_t hbytes = r->d_U ? 0 : r->ns * r->nt * sizeof(double);
      if (hbytes && !s->h_alloc.alloc(hbytes, &hoff)) break;
      if (!s->alloc.alloc(r->footprint, &off)) {
        if (hbytes) s->h_alloc.release(hoff, hbytes);
        break;
      }
      s->queue.pop_front();
      r->pool_off = off;
      r->h_off = hoff;
      s->pool_peak = std::max(s->pool_peak, s->alloc.used());
      const Clock::time_point h0 = Clock::now();
      g_srv_err.clear();
      int rc = start_req(s, *free_slot, r);
      s->host_seconds += std::chrono::duration<double>(Clock::now() - h0).count();
      if (rc) {
        const std::string msg = g_srv_err;
        // pending copies read the plan's host tables: wait for them, and keep
        // any error the stream reports
        const hipError_t se = hipStreamSynchronize(free_slot->st);
        drop_graph(*free_slot);
        s->alloc.release(off, r->footprint);
        if (hbytes) s->h_alloc.release(hoff, hbytes);
        free_slot->req = nullptr;
        free_slot->state = SL_IDLE;
        if (se != hipSuccess) {
          set_fatal(s, std::string("stream synchronization after a failed admission: ") + hipGetErrorString(se));
          g_srv_err = msg + "; " + s->fatal_msg;
          rc = PINT_EHIP;
        }
        if (rc == PINT_EHIP) set_fatal(s, msg);
        finish_req(s, r, rc);
      }
      progressed = true;
    }
    // progress of the active slots
    bool any_active = false;
    for (auto& sl : s->slots) {
      if (sl.state == SL_IDLE) continue;
      any_active = true;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      const Clock::time_point h0 = Clock::now();
      g_srv_err.clear();
      int rc = q == hipSuccess ? advance(s, sl)
                               : srv_fail(s, PINT_EHIP, std::string("stream error: ") + hipGetErrorString(q));
      s->host_seconds += std::chrono::duration<double>(Clock::now() - h0).count();
      if (rc) {
        Req* r = sl.req;
        const std::string msg = g_srv_err;
        const hipError_t se = hipStreamSynchronize(sl.st);
        if (se != hipSuccess) {
          rc = PINT_EHIP;
          g_srv_err = msg + "; stream synchronization: " + hipGetErrorString(se);
        }
        if (rc == PINT_EHIP) set_fatal(s, g_srv_err);
        drop_graph(sl);
        if (r) {
          s->alloc.release(r->pool_off, r->footprint);
          if (!r->d_U) s->h_alloc.release(r->h_off, r->ns * r->nt * sizeof(double));
          r->h_held = false;
          finish_req(s, r, rc);
        }
        sl.req = nullptr;
        sl.state = SL_IDLE;
      }
      progressed = true;
    }
    if (s->stop && !any_active && s->queue.empty()) break;
    if (!progressed) {
      if (any_active) {  // poll the slots' events again after letting submitters in
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
  }
}

// Shared part of the two submit calls: validate, build the plan, size the
// footprint, queue.  Exactly one of h_u0 and (d_u0, d_U) is given.
int submit_common(pint_server* s, const pint_problem* p, const double* h_u0, const double* d_u0, double* d_U,
                  uint64_t* ticket) {
  const Clock::time_point t_submit = Clock::now();  // latency includes plan construction
  pint_problem q = *p;
  q.flags |= PINT_FLAG_INIT_BROADCAST_U0;
  q.flags &= ~PINT_FLAG_STAGE_TIMING;
  PlanOpts o;
  o.host_mirror = false;
  o.defer_tables = true;
  pint_plan* plan = nullptr;
  int rc = plan_create_ex(&q, o, &plan);
  if (rc) return srv_fail(s, rc, std::string("invalid problem: ") + pint_last_error());
  Req* r = new (std::nothrow) Req();
  if (!r) {
    pint_plan_destroy(plan);
    return srv_fail(s, PINT_ENOMEM, "host allocation failed");
  }
  r->prob = q;
  r->plan = plan;
  r->ns = size_t(plan_ns(plan));
  r->nt = size_t(plan_nt(plan));
  r->tab_bytes = plan_table_bytes(&q);
  r->work_bytes = plan_workspace_bytes(plan);
  r->d_u0 = d_u0;
  r->d_U = d_U;
  if (d_U) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(d_U), b = reinterpret_cast<uintptr_t>(d_u0);
    const uintptr_t ua = a + r->ns * r->nt * sizeof(double), ub = b + r->ns * sizeof(double);
    if (a < ub && b < ua) {
      pint_plan_destroy(plan);
      delete r;
      return srv_fail(s, PINT_EINVAL, "d_u0 and d_U overlap");
    }
    r->footprint = al256(r->tab_bytes) + al256(r->work_bytes);
  } else {
    r->footprint = al256(r->tab_bytes) + al256(r->ns * 8) + al256(r->ns * r->nt * 8) + al256(r->work_bytes);
  }
  if (r->footprint > s->alloc.size()) {
    pint_plan_destroy(plan);
    delete r;
    return srv_fail(s, PINT_ENOMEM, "request footprint exceeds the whole pool");
  }
  if (!d_U && r->ns * r->nt * sizeof(double) > s->h_alloc.size()) {
    pint_plan_destroy(plan);
    delete r;
    return srv_fail(s, PINT_ENOMEM, "result exceeds the whole pinned host result pool");
  }
  if (h_u0) r->u0.assign(h_u0, h_u0 + r->ns);
  r->t_submit = t_submit;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal) {
      pint_plan_destroy(plan);
      delete r;
      return srv_fail(s, s->fatal, "server stopped after a HIP error: " + s->fatal_msg);
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    ++s->n_submitted;
  }
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return PINT_OK;
}

}  // namespace

extern "C" {

int pint_server_create(const pint_server_config* cfg, pint_server** out) {
  if (!out) return srv_fail(nullptr, PINT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || cfg->struct_size < sizeof(pint_server_config)) return srv_fail(nullptr, PINT_EINVAL, "bad config");
  if (!cfg->d_pool || cfg->pool_bytes < 4096) return srv_fail(nullptr, PINT_EINVAL, "pool missing or too small");
  if (reinterpret_cast<uintptr_t>(cfg->d_pool) % 256 != 0)
    return srv_fail(nullptr, PINT_EINVAL, "pool must be 256-byte aligned");
  const int nslots = cfg->max_active > 0 ? cfg->max_active : 8;
  if (nslots > 64) return srv_fail(nullptr, PINT_EINVAL, "max_active must be <= 64");
  pint_server* s = new (std::nothrow) pint_server();
  if (!s) return srv_fail(nullptr, PINT_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  s->pool = static_cast<unsigned char*>(cfg->d_pool);
  s->alloc.reset(cfg->pool_bytes & ~size_t(255));
  const size_t hbytes = cfg->host_pool_bytes ? cfg->host_pool_bytes : (size_t(1) << 30);
  if (hipHostMalloc(reinterpret_cast<void**>(&s->h_pool), hbytes, hipHostMallocDefault) != hipSuccess) {
    delete s;
    return srv_fail(nullptr, PINT_ENOMEM, "pinned host result pool allocation failed");
  }
  s->h_alloc.reset(hbytes & ~size_t(255));
  s->slots.resize(nslots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&sl.h_ctrl), sizeof(Ctrl), hipHostMallocCoherent) != hipSuccess) {
      pint_server_destroy(s);
      return srv_fail(nullptr, PINT_EHIP, "stream/event/pinned allocation failed");
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return PINT_OK;
}

int pint_server_submit(pint_server* s, const pint_problem* p, const double* h_u0, uint64_t* ticket) {
  if (!s || !p || !h_u0 || !ticket) return srv_fail(s, PINT_EINVAL, "NULL argument");
  return submit_common(s, p, h_u0, nullptr, nullptr, ticket);
}

int pint_server_submit_device(pint_server* s, const pint_problem* p, const double* d_u0, double* d_U,
                              uint64_t* ticket) {
  if (!s || !p || !d_u0 || !d_U || !ticket) return srv_fail(s, PINT_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_u0) % 8 || reinterpret_cast<uintptr_t>(d_U) % 8)
    return srv_fail(s, PINT_EINVAL, "device buffers must be 8-byte aligned");
  return submit_common(s, p, nullptr, d_u0, d_U, ticket);
}

int pint_server_wait(pint_server* s, uint64_t ticket, double* h_U, pint_report* rep, int timeout_ms) {
  if (!s) return srv_fail(nullptr, PINT_EINVAL, "server is NULL");
  if (rep && rep->struct_size < sizeof(pint_report)) return srv_fail(s, PINT_EINVAL, "report struct_size too small");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return srv_fail(s, PINT_ENOTFOUND, "unknown ticket");
  Req* r = it->second;
  if (r->waited) return srv_fail(s, PINT_EINVAL, "another thread is already waiting for this ticket");
  r->waited = true;
  auto ready = [&] { return r->state == RQ_DONE; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    r->waited = false;
    return srv_fail(s, PINT_ETIMEDOUT, "timed out");
  }
  const int status = r->status;
  s->reqs.erase(it);  // the request is ours now: copy out without holding the lock
  lk.unlock();
  if (r->h_held) {
    if (h_U) std::memcpy(h_U, s->h_pool + r->h_off, r->ns * r->nt * sizeof(double));
    lk.lock();
    s->h_alloc.release(r->h_off, r->ns * r->nt * sizeof(double));
    lk.unlock();
    s->cv_work.notify_one();  // freed result memory may admit a queued request
  }
  if (!r->err.empty() && status == r->status) g_srv_err = r->err;
  if (rep) {
    const size_t sz = rep->struct_size;
    *rep = r->rep;
    rep->struct_size = sz;
    rep->status = status;
  }
  delete r;
  return status;
}

int pint_server_cancel(pint_server* s, uint64_t ticket) {
  if (!s) return srv_fail(nullptr, PINT_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return srv_fail(s, PINT_ENOTFOUND, "unknown ticket");
    it->second->cancel = true;
  }
  s->cv_work.notify_one();
  return PINT_OK;
}

int pint_server_stats(pint_server* s, pint_server_statistics* st) {
  if (!s || !st || st->struct_size < sizeof(pint_server_statistics)) return srv_fail(s, PINT_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> g(s->mu);
  const size_t sz = st->struct_size;
  std::memset(st, 0, sizeof(pint_server_statistics));
  st->struct_size = sz;
  st->submitted = s->n_submitted;
  st->completed = s->n_completed;
  st->failed = s->n_failed;
  st->cancelled = s->n_cancelled;
  st->queued = int(s->queue.size());
  int active = 0;
  for (auto& sl : s->slots) active += sl.state != SL_IDLE;
  st->active = active;
  st->pool_bytes = s->alloc.size();
  st->pool_in_use = s->alloc.used();
  st->pool_peak = s->pool_peak;
  std::vector<double> l = s->lat_ms;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    const size_t i = size_t(q * double(l.size() - 1) + 0.5);
    return l[std::min(i, l.size() - 1)];
  };
  st->p50_ms = pct(0.50);
  st->p99_ms = pct(0.99);
  st->max_ms = l.empty() ? 0.0 : l.back();
  double sum = 0.0;
  for (double x : l) sum += x;
  st->mean_ms = l.empty() ? 0.0 : sum / double(l.size());
  st->dof_completed = s->dof_done;
  st->busy_seconds = s->have_first ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
  st->graphs_captured = s->graph_captures;
  st->graph_updates = s->graph_updates;
  st->graph_launches = s->graph_launches;
  st->worker_host_seconds = s->host_seconds;
  st->host_pool_bytes = s->h_alloc.size();
  st->host_pool_in_use = s->h_alloc.used();
  return PINT_OK;
}

int pint_server_destroy(pint_server* s) {
  if (!s) return PINT_OK;
  int rc = PINT_OK;
  std::string msg;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      for (Req* r : s->queue) r->cancel = true;
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
  }
  if (s->fatal != PINT_OK) {
    rc = s->fatal;
    msg = "server stopped after a HIP error: " + s->fatal_msg;
  }
  for (auto& sl : s->slots) {
    // a failure of the last work on a slot is reported here, not left for
    // the next unrelated synchronization to find
    if (sl.st) {
      const hipError_t e = hipStreamSynchronize(sl.st);
      if (e != hipSuccess && rc == PINT_OK) {
        rc = PINT_EHIP;
        msg = std::string("stream synchronization at shutdown: ") + hipGetErrorString(e);
      }
    }
    drop_graph(sl);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.h_ctrl) (void)hipHostFree(sl.h_ctrl);
    if (sl.h_in) (void)hipHostFree(sl.h_in);
  }
  for (auto& kv : s->reqs) {
    if (kv.second->plan) pint_plan_destroy(kv.second->plan);
    delete kv.second;
  }
  if (s->h_pool) (void)hipHostFree(s->h_pool);
  delete s;
  if (rc != PINT_OK) g_srv_err = msg;
  return rc;
}

const char* pint_server_last_error(const pint_server*) { return g_srv_err.c_str(); }

}  // extern "C"
