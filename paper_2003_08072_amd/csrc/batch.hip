// Many LPs at once: lp_solve_batch (a fixed set of handles) and the request
// server srv_* (a stream of LPs admitted by device-memory footprint).
//
// Both run each LP's IPM (Alg. 2) exactly as lp_solve does, on a stream of its
// own, from several host threads: the kernels of different LPs overlap on the
// device (the hardware queues interleave their workgroups), and the host-side
// control of one LP (stopping test, CG chunk checks, step read-back) never
// waits for another LP.  An LP's arithmetic does not depend on what runs beside
// it, so its result is bitwise the same alone and in a batch.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

namespace skipm {
void set_error(const std::string& msg);
}
using namespace skipm;

namespace {

int default_workers(int count) { return std::max(1, std::min(count, 8)); }

}  // namespace

extern "C" {

int lp_solve_batch(skipm_lp_t* lps, int32_t count, skipm_result* res, int32_t workers) {
  if (count < 0 || (count > 0 && (!lps || !res))) return set_error("null argument"), SKIPM_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!lps[i]) return set_error("null handle in batch"), SKIPM_EINVAL;
  if (count == 0) return SKIPM_OK;
  const int nw = workers > 0 ? std::min<int>(workers, count) : default_workers(count);
  // every handle's earlier work (create, reset, set_iterate on any stream) first
  SK_CHECK_HIP(hipDeviceSynchronize());
  int dev = 0;
  SK_CHECK_HIP(hipGetDevice(&dev));
  std::atomic<int> next{0};
  std::atomic<int> fatal{SKIPM_OK};
  std::mutex err_mu;
  std::string first_err;
  auto worker = [&]() {
    hipStream_t st = nullptr;
    if (hipSetDevice(dev) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      int expect = SKIPM_OK;
      fatal.compare_exchange_strong(expect, SKIPM_EDEVICE);
      return;
    }
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= count || fatal.load() != SKIPM_OK) break;
      const int rc = lp_solve(lps[i], &res[i], st);
      // ENOTCONV / ESTALL / ERANK / ENAN are outcomes of that LP (res[i].status);
      // argument and device errors end the batch
      if (rc == SKIPM_EINVAL || rc == SKIPM_EDEVICE || rc == SKIPM_ENOMEM) {
        int expect = SKIPM_OK;
        if (fatal.compare_exchange_strong(expect, rc)) {
          std::lock_guard<std::mutex> g(err_mu);
          first_err = skipm_last_error();
        }
        break;
      }
      if (res[i].status == SKIPM_OK && rc != SKIPM_OK) res[i].status = rc;
    }
    (void)hipStreamDestroy(st);
  };
  std::vector<std::thread> pool;
  pool.reserve(nw);
  for (int t = 0; t < nw; ++t) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  if (fatal.load() != SKIPM_OK) {
    set_error(first_err.empty() ? "device error in batch" : first_err);
    return fatal.load();
  }
  return SKIPM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the request server
// ---------------------------------------------------------------------------

struct skipm_server_s {
  struct Req {
    uint64_t ticket = 0;
    skipm_problem prob{};
    skipm_params prm{};
    double* x_out = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the producer stream at submit
    skipm_request_info info{};
  };
  int device = 0;
  int64_t budget = 0;
  int64_t in_use = 0, peak = 0;
  int32_t slots = 0, running = 0;
  int64_t completed = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::mutex mu;
  std::condition_variable work_cv;   // workers: a request may be admissible
  std::condition_variable done_cv;   // waiters: a request finished
  std::deque<Req*> queue;            // FIFO of admitted-later requests
  std::map<uint64_t, Req*> reqs;     // every request by ticket
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  bool head_fits() const {
    return !queue.empty() && queue.front()->info.footprint <= budget - in_use;
  }
  struct Outcome {
    skipm_result res{};
    int32_t rc = SKIPM_OK;
    int64_t device_bytes = 0;
  };
  void run(Req* r, hipStream_t st, Outcome* out);
  void worker_main();
};

// Runs one request.  The outcome goes to *out (a copy private to this
// worker); the caller publishes it into r->info under the lock, so srv_poll
// never sees a half-written result.
void skipm_server_s::run(Req* r, hipStream_t st, Outcome* out) {
  int rc = SKIPM_OK;
  if (r->ready && hipStreamWaitEvent(st, r->ready, 0) != hipSuccess) rc = SKIPM_EDEVICE;
  skipm_lp_t lp = nullptr;
  if (rc == SKIPM_OK) rc = lp_create(&lp, &r->prob, &r->prm, st);
  if (rc == SKIPM_OK) {
    rc = lp_solve(lp, &out->res, st);
    if (rc == SKIPM_ENOTCONV || rc == SKIPM_ESTALL || rc == SKIPM_ERANK || rc == SKIPM_ENAN)
      rc = SKIPM_OK;  // an outcome of the LP, in res.status
    if (rc == SKIPM_OK && r->x_out) rc = lp_get_iterate(lp, r->x_out, nullptr, nullptr, st);
    int64_t held = 0;
    lp_device_bytes(lp, &held);
    out->device_bytes = held;
  } else {
    out->res.status = rc;
  }
  if (lp) lp_destroy(lp);
  out->rc = rc;
}

void skipm_server_s::worker_main() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    std::unique_lock<std::mutex> lk(mu);
    work_cv.wait(lk, [&] { return (stop && queue.empty()) || (running < slots && head_fits()); });
    if (queue.empty()) break;  // stop requested and nothing left
    Req* r = queue.front();
    queue.pop_front();
    in_use += r->info.footprint;
    peak = std::max(peak, in_use);
    ++running;
    r->info.state = SKIPM_REQ_RUNNING;
    r->info.t_start = now();
    lk.unlock();
    Outcome oc;
    if (have_stream) {
      run(r, st, &oc);
    } else {
      oc.rc = SKIPM_EDEVICE;
      oc.res.status = SKIPM_EDEVICE;
    }
    lk.lock();
    r->info.res = oc.res;
    r->info.rc = oc.rc;
    r->info.device_bytes = oc.device_bytes;
    in_use -= r->info.footprint;
    --running;
    ++completed;
    r->info.t_done = now();
    r->info.state = SKIPM_REQ_DONE;
    if (r->ready) {
      (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
    }
    lk.unlock();
    work_cv.notify_all();
    done_cv.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

extern "C" {

int srv_create(skipm_server_t* out, int64_t hbm_budget, int32_t slots) {
  if (!out) return set_error("null argument"), SKIPM_EINVAL;
  *out = nullptr;
  if (hbm_budget <= 0) return set_error("hbm_budget must be positive"), SKIPM_EINVAL;
  if (slots < 1 || slots > 64) return set_error("slots must lie in [1, 64]"), SKIPM_EINVAL;
  auto* s = new skipm_server_s();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return set_error("hipGetDevice failed"), SKIPM_EDEVICE;
  }
  s->budget = hbm_budget;
  s->slots = slots;
  for (int i = 0; i < slots; ++i) s->workers.emplace_back([s] { s->worker_main(); });
  *out = s;
  return SKIPM_OK;
}

int srv_submit(skipm_server_t srv, const skipm_problem* prob, const skipm_params* prm,
               double* x_out, hipStream_t producer, uint64_t* ticket) {
  if (!srv || !prob || !prm || !ticket) return set_error("null argument"), SKIPM_EINVAL;
  int64_t fp = 0;
  SK_TRY(lp_footprint(prob, prm, &fp));
  if (fp > srv->budget)
    return set_error("request footprint " + std::to_string(fp) + " B exceeds the budget"),
           SKIPM_ENOMEM;
  auto* r = new skipm_server_s::Req();
  r->prob = *prob;
  r->prm = *prm;
  r->x_out = x_out;
  if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r->ready, producer) != hipSuccess) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    delete r;
    return set_error("could not record the producer event"), SKIPM_EDEVICE;
  }
  r->info.state = SKIPM_REQ_QUEUED;
  r->info.footprint = fp;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) {
      (void)hipEventDestroy(r->ready);
      delete r;
      return set_error("server is shutting down"), SKIPM_EINVAL;
    }
    r->ticket = srv->next_ticket++;
    r->info.t_submit = srv->now();
    srv->reqs[r->ticket] = r;
    srv->queue.push_back(r);
    *ticket = r->ticket;
  }
  srv->work_cv.notify_all();
  return SKIPM_OK;
}

int srv_poll(skipm_server_t srv, uint64_t ticket, skipm_request_info* info) {
  if (!srv || !info) return set_error("null argument"), SKIPM_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error("unknown ticket"), SKIPM_EINVAL;
  *info = it->second->info;
  return SKIPM_OK;
}

int srv_wait(skipm_server_t srv, uint64_t ticket, skipm_request_info* info) {
  if (!srv || !info) return set_error("null argument"), SKIPM_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error("unknown ticket"), SKIPM_EINVAL;
  skipm_server_s::Req* r = it->second;
  srv->done_cv.wait(lk, [&] { return r->info.state == SKIPM_REQ_DONE; });
  *info = r->info;
  return SKIPM_OK;
}

int srv_now(skipm_server_t srv, double* t) {
  if (!srv || !t) return set_error("null argument"), SKIPM_EINVAL;
  *t = srv->now();
  return SKIPM_OK;
}

int srv_stats(skipm_server_t srv, skipm_server_stats* out) {
  if (!srv || !out) return set_error("null argument"), SKIPM_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  out->budget = srv->budget;
  out->in_use = srv->in_use;
  out->peak_in_use = srv->peak;
  out->slots = srv->slots;
  out->running = srv->running;
  out->queued = (int32_t)srv->queue.size();
  out->completed = srv->completed;
  return SKIPM_OK;
}

int srv_destroy(skipm_server_t srv) {
  if (!srv) return SKIPM_OK;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->work_cv.notify_all();
  for (auto& th : srv->workers) th.join();
  for (auto& kv : srv->reqs) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  delete srv;
  return SKIPM_OK;
}

}  // extern "C"
