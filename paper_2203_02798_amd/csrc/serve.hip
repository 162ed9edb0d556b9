// Request server of libpsk: continuous batching of least-squares and
// leverage-score requests on one GPU.
//
// Paper mapping (arXiv 2203.02798): each request is one run of Algorithm
// least_squares_precondition (lsq_solve) or of the sketched leverage scores
// of Algorithm ls_approximate_drineas (sketch_gcs, sketch_qr, rownorms_sq on
// A R^{-1}); the server only schedules them.
//
// Design: `slots` worker threads, each with its own HIP stream, take
// requests in arrival order.  A request is admitted when a slot is free and
// its whole workspace (sized by the same dry run as psk_workspace_size) fits
// in the caller's device pool; the pool is carved by a first-fit allocator
// with coalescing, so the device-memory footprint of the requests in flight
// never exceeds the pool.  Admission is strictly first-in first-out (a large
// request at the head waits for memory rather than being overtaken).
// Requests on different slots overlap on the device; each request's kernels
// read only its own inputs and workspace, so its result does not depend on
// what else runs.
#include <math.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "server_book.hpp"

namespace psk {
namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
  psk_request req;
  int64_t ticket = 0;
  size_t ws_bytes = 0;
  size_t ws_off = SIZE_MAX;
  double t_submit = 0, t_start = 0, t_end = 0;
  int status = PSK_OK;
  psk_lsq_info info{};
  bool done = false;
};

// A leverage request: leverage_sketch without the JL step and without the
// rank check (which would synchronise the slot's stream mid-request).
int leverage_run(const psk_request &q, Arena &ws, hipStream_t st) {
  return leverage_sketch_impl(q.A, q.opts.m, q.opts.r, 0, q.opts.seed, q.opts.prec, q.out,
                              false, ws, st);
}

int plan_request(const psk_request &q, size_t *bytes) {
  Arena plan;
  int rc = validate_csr(q.A, plan, nullptr);
  if (rc) return rc;
  if (q.op == PSK_REQ_LSQ) {
    rc = lsq_impl(q.A, nullptr, nullptr, q.opts, nullptr, plan, nullptr);
  } else {
    rc = leverage_run(q, plan, nullptr);
  }
  if (rc) return rc;
  *bytes = plan.peak + kAlign;
  return 0;
}

}  // namespace

struct Server {
  int device = 0;
  unsigned char *pool = nullptr;
  size_t pool_bytes = 0;
  PoolAlloc alloc{0};
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work;
  std::deque<Job *> queue;
  TicketBoard<Job> jobs;
  int inflight = 0, inflight_peak = 0;
  int64_t submitted = 0, completed = 0;
  bool stop = false;

  void worker(int slot) {
    (void)hipSetDevice(device);
    hipStream_t st = streams[slot];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      Job *job = nullptr;
      cv_work.wait(lk, [&] {
        if (stop && queue.empty()) return true;
        if (queue.empty()) return false;
        const size_t off = alloc.alloc(queue.front()->ws_bytes);
        if (off == SIZE_MAX) return false;
        queue.front()->ws_off = off;
        return true;
      });
      if (queue.empty()) return;  // stopping and nothing left
      job = queue.front();
      queue.pop_front();
      ++inflight;
      if (inflight > inflight_peak) inflight_peak = inflight;
      job->t_start = now_s();
      lk.unlock();
      cv_work.notify_all();  // the next request may fit as well
      Arena ws = Arena::over(pool + job->ws_off, job->ws_bytes);
      // a malformed CSR A ends the request before any kernel walks it
      int rc = validate_csr(job->req.A, ws, st);
      if (!rc)
        rc = job->req.op == PSK_REQ_LSQ ? lsq_impl(job->req.A, job->req.b, job->req.out,
                                                   job->req.opts, &job->info, ws, st)
                                        : leverage_run(job->req, ws, st);
      const hipError_t e = hipStreamSynchronize(st);
      if (!rc && e != hipSuccess) rc = fail(PSK_EDEVICE, hipGetErrorString(e));
      lk.lock();
      job->status = rc;
      job->t_end = now_s();
      job->done = true;
      alloc.release(job->ws_off);
      --inflight;
      ++completed;
      jobs.completed();
      cv_work.notify_all();
    }
  }
};

}  // namespace psk

using namespace psk;

extern "C" {

int psk_server_create(const psk_server_opts *o, psk_server **out) {
  if (!o || !out) return fail(PSK_EINVAL, "NULL argument");
  if (o->slots < 1 || o->slots > 64) return fail(PSK_EINVAL, "slots must be in [1, 64]");
  if (!o->pool || o->pool_bytes < kAlign)
    return fail(PSK_EINVAL, "a device pool of at least 256 bytes is needed");
  if (((uintptr_t)o->pool % kAlign) != 0)
    return fail(PSK_EINVAL, "the pool must be 256-byte aligned");
  Server *s = new Server();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(PSK_EDEVICE, "hipGetDevice failed");
  }
  s->pool = (unsigned char *)o->pool;
  s->pool_bytes = o->pool_bytes;
  s->alloc = PoolAlloc(o->pool_bytes);
  for (int i = 0; i < o->slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return fail(PSK_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < o->slots; ++i) s->workers.emplace_back([s, i] { s->worker(i); });
  *out = reinterpret_cast<psk_server *>(s);
  return PSK_OK;
}

int psk_server_submit(psk_server *srv, const psk_request *q, int64_t *ticket) {
  if (!srv || !q || !ticket) return fail(PSK_EINVAL, "NULL argument");
  Server *s = reinterpret_cast<Server *>(srv);
  int rc = check_mat(&q->A);
  if (rc) return rc;
  if (q->op != PSK_REQ_LSQ && q->op != PSK_REQ_LEVERAGE)
    return fail(PSK_EINVAL, "op must be PSK_REQ_LSQ or PSK_REQ_LEVERAGE");
  if (!q->out) return fail(PSK_EINVAL, "out is NULL");
  const psk_lsq_opts &o = q->opts;
  if (q->op == PSK_REQ_LSQ) {
    if (!q->b) return fail(PSK_EINVAL, "b is NULL");
    if (!o.Rinv) {
      if (o.m < q->A.d) return fail(PSK_EINVAL, "opts.m must be >= d");
      if ((rc = check_r(o.r))) return rc;
      if (o.r < o.m) return fail(PSK_EINVAL, "opts.r must be >= opts.m");
    }
    if (o.max_iter < 1 || o.check_every < 1 || o.refine < 0)
      return fail(PSK_EINVAL, "max_iter >= 1, check_every >= 1, refine >= 0 needed");
  } else {
    if (o.m < q->A.d) return fail(PSK_EINVAL, "opts.m must be >= d");
    if ((rc = check_r(o.r))) return rc;
    if (o.r < o.m) return fail(PSK_EINVAL, "opts.r must be >= opts.m");
  }
  if (o.prec != PSK_PREC_F64 && o.prec != PSK_PREC_BF16 && o.prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "opts.prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  size_t bytes = 0;
  if ((rc = plan_request(*q, &bytes))) return rc;
  if (bytes > s->pool_bytes)
    return fail(PSK_ENOMEM, "request workspace exceeds the whole server pool");
  Job *job = new Job();
  job->req = *q;
  job->ws_bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete job;
      return fail(PSK_EINVAL, "server is shutting down");
    }
    job->t_submit = now_s();
    job->ticket = s->jobs.add(job);
    s->queue.push_back(job);
    ++s->submitted;
  }
  s->cv_work.notify_all();
  *ticket = job->ticket;
  return PSK_OK;
}

static void fill_result(const Job *j, psk_result *res) {
  res->status = j->status;
  res->iters = j->info.iters;
  res->resid = j->info.resid;
  res->ne_resid = j->info.ne_resid;
  res->t_submit = j->t_submit;
  res->t_start = j->t_start;
  res->t_end = j->t_end;
  res->prec_used = j->req.op == PSK_REQ_LSQ ? j->info.prec_used : j->req.opts.prec;
  res->reserved = 0;
  res->delta_est = j->req.op == PSK_REQ_LSQ ? j->info.delta_est : NAN;
}

static int ticket_status(int rc) {
  if (rc == TicketBoard<Job>::kUnknown) return fail(PSK_EINVAL, "unknown ticket");
  if (rc == TicketBoard<Job>::kClaimed)
    return fail(PSK_EINVAL, "another thread is already waiting for this ticket");
  return rc == TicketBoard<Job>::kPending ? PSK_PENDING : PSK_OK;
}

int psk_server_wait(psk_server *srv, int64_t ticket, psk_result *res) {
  if (!srv || !res) return fail(PSK_EINVAL, "NULL argument");
  Server *s = reinterpret_cast<Server *>(srv);
  std::unique_lock<std::mutex> lk(s->mu);
  return ticket_status(s->jobs.wait(lk, ticket, [&](const Job &j) { fill_result(&j, res); }));
}

int psk_server_poll(psk_server *srv, int64_t ticket, psk_result *res) {
  if (!srv || !res) return fail(PSK_EINVAL, "NULL argument");
  Server *s = reinterpret_cast<Server *>(srv);
  std::lock_guard<std::mutex> lk(s->mu);
  return ticket_status(s->jobs.poll(ticket, [&](const Job &j) { fill_result(&j, res); }));
}

int psk_server_stats(psk_server *srv, psk_server_stats_t *out) {
  if (!srv || !out) return fail(PSK_EINVAL, "NULL argument");
  Server *s = reinterpret_cast<Server *>(srv);
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->queued = (int64_t)s->queue.size();
  out->inflight = s->inflight;
  out->inflight_peak = s->inflight_peak;
  out->pool_bytes = s->pool_bytes;
  out->pool_used = s->alloc.used();
  out->pool_peak = s->alloc.peak();
  return PSK_OK;
}

int psk_server_destroy(psk_server *srv) {
  if (!srv) return fail(PSK_EINVAL, "NULL argument");
  Server *s = reinterpret_cast<Server *>(srv);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  s->jobs.clear();
  delete s;
  return PSK_OK;
}

}  // extern "C"
