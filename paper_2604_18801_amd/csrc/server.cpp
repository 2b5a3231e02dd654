// Served form of the correction pass: a job queue in front of the batched
// pipeline, drained by slot threads that each own a context (workspace and
// HIP stream) on the same device, and one shared PGD loop (engine.cpp).  A
// slot takes the queued jobs in arrival order, as many as fit its share of
// the device memory, and prepares them on its own stream (every stage up to
// the first PGD step); their PGD state then joins the shared loop, which
// steps every resident call's jobs in the same launches and lets each call
// leave as soon as its jobs have converged, when its slot encodes them and
// takes the next jobs.  Jobs are thus admitted and retired at the
// granularity of a few PGD steps (iteration-level continuous batching),
// and the setup and encoding of some calls overlap the iterations of
// others on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.hpp"

namespace {

using Clock = std::chrono::steady_clock;

enum : int { kQueued = 0, kRunning = 1, kDone = 2 };

struct Rec {
  pcc_job job;
  pcc_job_result res;
  int state = kQueued;
  bool solo = false;  // run alone (after its batch ran out of memory)
  bool retried = false;  // ran out of memory alone once already
  size_t footprint = 0;  // workspace bound from pcc_workspace_query (0: not known)
  std::string err;
};

// device bytes per particle assumed for admission until a batch of at least
// kLearnMin particles has been measured
constexpr double kBytesPerParticle0 = 2048.0;
constexpr int64_t kLearnMin = 100000;
// jobs at least this large are admitted by their counted footprint
// (pcc_workspace_query on the slot's stream), the others by the estimate
constexpr int64_t kQueryMin = 1000000;

}  // namespace

struct pcc_server {
  int device = 0;
  pcc::PgdEngine *engine = nullptr;  // the shared PGD loop
  double budget = 0.0;
  int max_inflight = 256;
  std::vector<pcc_context *> ctx;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Rec> recs;
  uint64_t next = 1;
  size_t outstanding = 0;
  bool stop = false;
  double bpp = kBytesPerParticle0;
  double reserved = 0.0;  // workspace bytes the running calls hold
  Clock::time_point t0 = Clock::now();

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
};

namespace {

pcc_status fail(pcc_status s, const std::string &m) {
  pcc::set_last_error(m);
  return s;
}

bool needs_query(const Rec &r) { return r.footprint == 0 && r.job.orig.n >= kQueryMin; }

double footprint_of(const pcc_server *S, const Rec &r) {
  return r.footprint ? (double)r.footprint : (double)std::max<int64_t>(r.job.orig.n, 1) * S->bpp;
}

// Admission: jobs in arrival order while the device memory not held by the
// running calls covers their footprints (counted for large jobs, estimated
// for the others).  A job that does not fit waits for memory to free up,
// unless nothing is running (then it is taken and may run out of memory).
// A job whose footprint is still to be counted is taken alone.
void take_batch(pcc_server *S, std::vector<uint64_t> &batch, double &est) {
  est = 0.0;
  while (!S->queue.empty() && (int)batch.size() < S->max_inflight) {
    const uint64_t tk = S->queue.front();
    Rec &r = S->recs[tk];
    const bool count = needs_query(r);
    const double e = footprint_of(S, r);
    if (!batch.empty() && (r.solo || count || S->reserved + est + e > S->budget)) break;
    if (batch.empty() && !count && S->reserved > 0.0 && S->reserved + e > S->budget) break;
    S->queue.pop_front();
    r.state = kRunning;
    r.res.t_start_ms = S->now_ms();
    batch.push_back(tk);
    est += e;
    if (r.solo || count) break;
  }
}

void worker_main(pcc_server *S, int w) {
  hipSetDevice(S->device);
  pcc::Context &C = S->ctx[w]->c;
  std::vector<uint64_t> batch;
  std::vector<pcc_job> jobs;
  std::vector<pcc_job_result> res;
  for (;;) {
    batch.clear();
    double hold = 0.0;  // workspace bytes this call reserves
    bool count = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->queue.empty()) return;  // stopping, nothing left
      take_batch(S, batch, hold);
      if (batch.empty()) {
        // the next job waits for memory held by running calls
        S->cv_work.wait(lk);
        continue;
      }
      count = batch.size() == 1 && needs_query(S->recs[batch[0]]);
      if (!count) S->reserved += hold;
      jobs.clear();
      for (uint64_t tk : batch) jobs.push_back(S->recs[tk].job);
    }
    res.assign(batch.size(), pcc_job_result{});
    pcc_status err = PCC_OK;
    std::string msg;
    if (count) {
      // count the large job's footprint on this slot's stream, then admit
      // it by that (or put it back until memory frees up)
      size_t fp = 0;
      try {
        pcc_job_result q{};
        pcc::run_batch(C, jobs.data(), 1, &q, C.own, false, false, nullptr, &fp);
      } catch (const std::exception &) {
        fp = 0;  // the correction itself reports the failure
      }
      std::unique_lock<std::mutex> lk(S->mu);
      Rec &r = S->recs[batch[0]];
      r.footprint = fp ? fp : (size_t)footprint_of(S, r) + 1;
      hold = (double)r.footprint;
      if (S->reserved > 0.0 && S->reserved + hold > S->budget) {
        r.state = kQueued;
        S->queue.push_front(batch[0]);
        S->cv_work.notify_all();
        continue;
      }
      S->reserved += hold;
    }
    try {
      pcc::run_batch(C, jobs.data(), (int)jobs.size(), res.data(), C.own, false);
    } catch (const pcc::Error &e) {
      err = e.status;
      msg = e.what();
    } catch (const std::bad_alloc &) {
      err = PCC_E_OUT_OF_MEMORY;
      msg = "host allocation failed";
    } catch (const std::exception &e) {
      err = PCC_E_DEVICE;
      msg = e.what();
    }
    // a workspace grown beyond the slot's share of the budget goes back to
    // the device (so that idle slots do not hold what running ones need);
    // after running out of memory the next batch starts afresh
    if (err == PCC_E_OUT_OF_MEMORY || (double)C.arena.capacity() > S->budget / (double)S->ctx.size())
      C.arena.release();
    std::lock_guard<std::mutex> lk(S->mu);
    S->reserved -= hold;
    S->cv_work.notify_all();  // memory freed: a waiting job may fit now
    if (err == PCC_E_OUT_OF_MEMORY && (batch.size() > 1 || !S->recs[batch[0]].retried)) {
      // run each job of the batch on its own, at the head of the queue; a
      // job that ran out of memory alone gets one more try with the
      // worker's workspace released
      const bool alone = batch.size() == 1;
      for (auto it = batch.rbegin(); it != batch.rend(); ++it) {
        Rec &r = S->recs[*it];
        r.state = kQueued;
        r.solo = true;
        r.retried |= alone;
        S->queue.push_front(*it);
      }
      S->cv_work.notify_all();
      continue;
    }
    int64_t np = 0;
    for (const pcc_job &j : jobs) np += j.orig.n;
    if (err == PCC_OK && np >= kLearnMin)
      S->bpp = std::max(S->bpp, (double)C.arena.used() / (double)np);
    const double tf = S->now_ms();
    for (size_t k = 0; k < batch.size(); ++k) {
      Rec &r = S->recs[batch[k]];
      const double ts = r.res.t_submit_ms, tb = r.res.t_start_ms;
      if (err == PCC_OK) {
        r.res = res[k];
      } else {
        std::memset(&r.res, 0, sizeof r.res);
        r.res.status = err;
        r.err = msg;
      }
      r.res.t_submit_ms = ts;
      r.res.t_start_ms = tb;
      r.res.t_finish_ms = tf;
      r.res.batch_jobs = (int32_t)batch.size();
      r.res.worker = w;
      r.state = kDone;
      --S->outstanding;
    }
    S->cv_done.notify_all();
  }
}

pcc_status result_of(const Rec &r, pcc_job_result *out) {
  if (r.state != kDone) {
    if (out) {
      *out = r.res;
      out->status = PCC_PENDING;
    }
    return PCC_PENDING;
  }
  if (out) *out = r.res;
  if (r.res.status < 0) pcc::set_last_error(r.err.empty() ? pcc_status_string(r.res.status) : r.err);
  return r.res.status;
}

}  // namespace

extern "C" {

pcc_status pcc_server_create(pcc_context *ctx, const pcc_server_config *cfg, pcc_server **out) {
  if (!ctx || !out) return fail(PCC_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  pcc_server_config c{};
  if (cfg) c = *cfg;
  if (c.max_inflight < 0 || c.max_inflight > PCC_MAX_BATCH_JOBS || c.n_streams < 0 ||
      c.n_streams > 32)
    return fail(PCC_E_INVALID_ARG, "max_inflight >= 0 and n_streams in 0..32");
  try {
    auto *S = new pcc_server;
    S->device = ctx->c.device;
    S->max_inflight = c.max_inflight ? c.max_inflight : 256;
    const int nw = c.n_streams ? c.n_streams : 16;
    if (hipSetDevice(S->device) != hipSuccess) {
      delete S;
      return fail(PCC_E_DEVICE, "hipSetDevice failed");
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete S;
      return fail(PCC_E_DEVICE, "hipMemGetInfo failed");
    }
    S->budget = c.hbm_budget ? (double)c.hbm_budget : 0.8 * (double)free_b;
    try {
      S->engine = pcc::engine_create(S->device, ctx->c.graph_iters);
    } catch (const pcc::Error &e) {
      delete S;
      return fail(e.status, e.what());
    }
    for (int w = 0; w < nw; ++w) {
      pcc_context *h = nullptr;
      const pcc_status st = pcc_context_create(S->device, &h);
      if (st != PCC_OK) {
        for (auto *x : S->ctx) pcc_context_destroy(x);
        pcc::engine_destroy(S->engine);
        delete S;
        return st;
      }
      h->c.engine = S->engine;
      h->c.graph_iters = ctx->c.graph_iters;
      h->c.cell_pct = ctx->c.cell_pct;
      h->c.dense_cell = ctx->c.dense_cell;
      h->c.force_exact_pairs = ctx->c.force_exact_pairs;
      S->ctx.push_back(h);
    }
    for (int w = 0; w < nw; ++w) S->workers.emplace_back(worker_main, S, w);
    *out = S;
    return PCC_OK;
  } catch (const std::exception &e) {
    return fail(PCC_E_OUT_OF_MEMORY, e.what());
  }
}

pcc_status pcc_server_submit(pcc_server *srv, const pcc_job *job, uint64_t *ticket) {
  if (!srv || !job || !ticket) return fail(PCC_E_INVALID_ARG, "NULL argument");
  if (job->orig.n < 0 || job->orig.n != job->recon.n)
    return fail(PCC_E_INVALID_ARG, "orig and recon must have the same n >= 0");
  try {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(PCC_E_INVALID_ARG, "server is shutting down");
    const uint64_t tk = srv->next++;
    Rec &r = srv->recs[tk];
    r.job = *job;
    std::memset(&r.res, 0, sizeof r.res);
    r.res.status = PCC_PENDING;
    r.res.t_submit_ms = srv->now_ms();
    srv->queue.push_back(tk);
    ++srv->outstanding;
    *ticket = tk;
  } catch (const std::exception &e) {
    return fail(PCC_E_OUT_OF_MEMORY, e.what());
  }
  srv->cv_work.notify_one();
  return PCC_OK;
}

pcc_status pcc_server_poll(pcc_server *srv, uint64_t ticket, pcc_job_result *result) {
  if (!srv) return fail(PCC_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->recs.find(ticket);
  if (it == srv->recs.end()) return fail(PCC_E_INVALID_ARG, "unknown ticket");
  return result_of(it->second, result);
}

pcc_status pcc_server_wait(pcc_server *srv, uint64_t ticket, int64_t timeout_ms,
                           pcc_job_result *result) {
  if (!srv) return fail(PCC_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->recs.find(ticket);
  if (it == srv->recs.end()) return fail(PCC_E_INVALID_ARG, "unknown ticket");
  Rec &r = it->second;
  auto done = [&] { return r.state == kDone; };
  if (timeout_ms < 0)
    srv->cv_done.wait(lk, done);
  else
    srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
  return result_of(r, result);
}

pcc_status pcc_server_cancel(pcc_server *srv, uint64_t ticket) {
  if (!srv) return fail(PCC_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->recs.find(ticket);
  if (it == srv->recs.end() || it->second.state != kQueued)
    return fail(PCC_E_INVALID_ARG, "unknown ticket, or the job has started");
  auto q = std::find(srv->queue.begin(), srv->queue.end(), ticket);
  if (q != srv->queue.end()) srv->queue.erase(q);
  Rec &r = it->second;
  r.state = kDone;
  r.res.status = PCC_E_CANCELLED;
  r.res.t_finish_ms = srv->now_ms();
  r.err = "cancelled";
  --srv->outstanding;
  srv->cv_done.notify_all();
  return PCC_OK;
}

pcc_status pcc_server_drain(pcc_server *srv) {
  if (!srv) return fail(PCC_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
  return PCC_OK;
}

pcc_status pcc_server_destroy(pcc_server *srv) {
  if (!srv) return PCC_OK;
  pcc_server_drain(srv);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto &t : srv->workers) t.join();
  pcc::engine_destroy(srv->engine);
  for (auto *c : srv->ctx) pcc_context_destroy(c);
  delete srv;
  return PCC_OK;
}

}  // extern "C"
