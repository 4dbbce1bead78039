// Many LPs at once: lp_solve_batch (a fixed set of handles) and the request
// server srv_* (a stream of LPs admitted by device-memory footprint).
//
// Both run each LP's IPM (Alg. 2) exactly as lp_solve does, on a stream of its
// own, from several host threads: the kernels of different LPs overlap on the
// device (the hardware queues interleave their workgroups), and the host-side
// control of one LP (stopping test, CG chunk checks, step read-back) never
// waits for another LP.  An LP's arithmetic does not depend on what runs beside
// it, so its result is bitwise the same alone and in a batch.
#include <string.h>

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
#include "handle.h"

using namespace skipm;

namespace {

int default_workers(int count) { return std::max(1, std::min(count, 8)); }

// ---------------------------------------------------------------------------
// The grouped engine for the dense FP64-product LPs of a batch.  Each LP runs
// its own IPM iterations; what is grouped is the CG, the hot loop:
//   - host workers (one stream each) take an LP through the start of an
//     iteration (stopping test, sketch, Gram factorisation; the CG too if it
//     runs in one workgroup) and, after its CG, through the end (rank-loss
//     retries, epilogue, correction vector, step), then straight into the
//     start of its next iteration;
//   - one executor runs the CG of every LP that is ready, in grouped
//     launches: per CG iteration one launch per pass and lane-group shape
//     (product pass, finish, Q^{-1} pass), whose work list is the (LP,
//     workgroup) pairs of its LPs.  Every LP keeps the workgroup count,
//     column ranges, partial sums and CG iteration index of its own launches,
//     so its arithmetic is that of a lone solve.  LPs join the launches when
//     their set-up is done and leave them at the host check after their done
//     flag is set (their workgroups return at once until then); the host
//     reads all flags once per chunk of iterations.
// ---------------------------------------------------------------------------

struct Group {
  ColKey key;
  std::vector<int> members;    // positions in the staged LP list
  std::vector<int32_t> first;  // workgroup offsets, members.size() + 1
  size_t args_off = 0, first_off = 0, kst_off = 0;
};

// The CG arguments of one LP, prepared once per batch.
struct CgPrep {
  bool ready = false;
  ColKey kn, kd;
  int nb_n = 0, nb_c = 0, nb_q = 0, fnb = 0;
  std::vector<char> a_n, a_c, a_q;  // argument blocks: 2 (parities), 2, 1
  FinishDotArgs fin[2];
  CgInitArgs init;
  int32_t* is = nullptr;
};

std::vector<Group> group_by(const std::vector<ColKey>& keys, const std::vector<int>& nb) {
  std::vector<Group> out;
  for (int i = 0; i < (int)keys.size(); ++i) {
    Group* g = nullptr;
    for (auto& h : out)
      if (h.key == keys[i]) g = &h;
    if (!g) {
      out.emplace_back();
      g = &out.back();
      g->key = keys[i];
      g->first.push_back(0);
    }
    g->members.push_back(i);
    g->first.push_back(g->first.back() + nb[i]);
  }
  return out;
}

constexpr int kChunk = 6;  // CG iterations between host checks of the grouped CG

class Engine {
 public:
  Engine(skipm_lp_t* lps, skipm_result* res, std::vector<int> idx, int nthreads, int dev)
      : lps_(lps), res_(res), idx_(std::move(idx)), nthreads_(nthreads), dev_(dev) {}

  ~Engine() {
    if (dbuf_) (void)hipFree(dbuf_);
    if (hbuf_) (void)hipHostFree(hbuf_);
    if (hflags_) (void)hipHostFree(hflags_);
  }

  int run(std::string* err) {
    if (hipSetDevice(dev_) != hipSuccess) return *err = "hipSetDevice failed", SKIPM_EDEVICE;
    const int n = (int)idx_.size();
    st_.assign(n, BatchLp{});
    prep_.assign(n, CgPrep{});
    for (int i : idx_) memset(&res_[i], 0, sizeof(res_[i]));
    ab_ = colpass_args_bytes();
    int rc = SKIPM_OK;
    if (hipStreamCreateWithFlags(&cg_st_, hipStreamNonBlocking) != hipSuccess) {
      *err = "could not create the batch's streams";
      return SKIPM_EDEVICE;
    }
    streams_.assign(nthreads_, nullptr);
    for (auto& s : streams_)
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        rc = SKIPM_EDEVICE;
        *err = "could not create the batch's streams";
      }
    if (rc == SKIPM_OK) {
      outstanding_ = n;
      for (int q = 0; q < n; ++q) tasks_.push_back({q, false});
      std::vector<std::thread> pool;
      for (int t = 0; t < nthreads_; ++t) pool.emplace_back([this, t] { worker(t); });
      rc = execute();
      {
        std::lock_guard<std::mutex> g(mu_);
        stop_ = true;
      }
      cv_.notify_all();
      for (auto& th : pool) th.join();
      if (rc == SKIPM_OK && fatal_ != SKIPM_OK) rc = fatal_;
      *err = rc == SKIPM_OK ? "" : (fatal_ != SKIPM_OK ? fatal_msg_ : skipm_last_error());
    }
    for (auto& s : streams_)
      if (s) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(cg_st_);
    return rc;
  }

 private:
  struct Task {
    int q;          // position in idx_
    bool after_cg;  // run the end of the iteration first
  };

  void worker(int t) {
    (void)hipSetDevice(dev_);
    hipStream_t s = streams_[t];
    for (;;) {
      Task task;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || !tasks_.empty(); });
        if (tasks_.empty()) return;
        task = tasks_.front();
        tasks_.pop_front();
      }
      skipm_lp_s* lp = lps_[idx_[task.q]];
      skipm_result* res = &res_[idx_[task.q]];
      BatchLp* b = &st_[task.q];
      if (task.after_cg) {
        batch_phase_b(lp, res, b, s);
        (void)hipStreamSynchronize(s);
      }
      if (b->active) {
        batch_phase_a(lp, res, b, s);
        (void)hipStreamSynchronize(s);
      }
      std::lock_guard<std::mutex> g(mu_);
      if (b->rc != SKIPM_OK && fatal_ == SKIPM_OK) {
        fatal_ = b->rc;
        fatal_msg_ = b->err;
      }
      if (!b->active) {
        --outstanding_;
      } else if (b->grouped) {
        ready_.push_back(task.q);
      } else {
        tasks_.push_back({task.q, true});  // its CG ran in one workgroup
      }
      cv_.notify_all();
    }
  }

  // The executor: the grouped CG of the LPs that are ready, chunk by chunk.
  int execute() {
    std::vector<int> in_cg;        // positions in idx_
    std::vector<int64_t> kstart;   // their next CG iteration
    for (;;) {
      std::vector<int> fresh;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (in_cg.empty())
          cv_.wait(lk, [&] { return !ready_.empty() || outstanding_ == 0 || fatal_ != SKIPM_OK; });
        if (fatal_ != SKIPM_OK) return fatal_;
        if (in_cg.empty() && ready_.empty() && outstanding_ == 0) return SKIPM_OK;
        fresh.assign(ready_.begin(), ready_.end());
        ready_.clear();
      }
      if (!fresh.empty()) {
        for (int q : fresh) SK_TRY(prepare(q));
        // CG set-up of the newcomers: z_0 = Q^{-1} p, then r, z, d, x and the
        // stopping threshold
        SK_TRY(stage(fresh, nullptr, true));
        for (auto& g : gq_)
          if (launch_colpass_grouped(g.key, dp(g.args_off), (const int32_t*)dp(g.first_off),
                                     (int)g.members.size(), g.first.back(), nullptr, 0, cg_st_) != 0)
            return set_error("grouped CG: no kernel for a shape"), SKIPM_EINVAL;
        launch_cg_init_grouped((const CgInitArgs*)dp(init_off_), (int)fresh.size(), cg_st_);
        SK_CHECK_HIP(hipGetLastError());
        for (int q : fresh) {
          in_cg.push_back(q);
          kstart.push_back(0);
        }
        SK_CHECK_HIP(hipStreamSynchronize(cg_st_));  // the staging buffer is reused below
      }
      if (in_cg.empty()) continue;
      SK_TRY(stage(in_cg, &kstart, false));
      const int na = (int)in_cg.size();
      const int64_t* ks = (const int64_t*)dp(kstart_off_);
      for (int j = 0; j < kChunk; ++j) {
        for (auto& g : gn_)
          if (launch_colpass_grouped(g.key, dp(g.args_off), (const int32_t*)dp(g.first_off),
                                     (int)g.members.size(), g.first.back(),
                                     (const int64_t*)dp(g.kst_off), j, cg_st_) != 0)
            return set_error("grouped CG: no kernel for a shape"), SKIPM_EINVAL;
        launch_finish_dot_grouped((const FinishDotArgs*)dp(fin_off_), (const int32_t*)dp(ffirst_off_),
                                  na, ffirst_.back(), ks, j, cg_st_);
        for (auto& g : gd_)
          if (launch_colpass_grouped(g.key, dp(g.args_off), (const int32_t*)dp(g.first_off),
                                     (int)g.members.size(), g.first.back(),
                                     (const int64_t*)dp(g.kst_off), j, cg_st_) != 0)
            return set_error("grouped CG: no kernel for a shape"), SKIPM_EINVAL;
      }
      launch_cg_flags((int32_t* const*)dp(isp_off_), na, (int32_t*)dp(flags_off_), cg_st_);
      SK_CHECK_HIP(hipGetLastError());
      SK_CHECK_HIP(hipMemcpyAsync(hflags_, dp(flags_off_), 3 * na * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, cg_st_));
      SK_CHECK_HIP(hipStreamSynchronize(cg_st_));
      std::vector<int> keep;
      std::vector<int64_t> kkeep;
      std::vector<int> finished;
      for (int q = 0; q < na; ++q) {
        const int p = in_cg[q];
        if (hflags_[3 * q]) {
          st_[p].its = hflags_[3 * q + 1];
          st_[p].fail = hflags_[3 * q + 2] ? 1 : 0;
          finished.push_back(p);
        } else {
          keep.push_back(p);
          kkeep.push_back(kstart[q] + kChunk);
        }
      }
      in_cg.swap(keep);
      kstart.swap(kkeep);
      if (!finished.empty()) {
        std::lock_guard<std::mutex> g(mu_);
        for (int p : finished) tasks_.push_back({p, true});
        cv_.notify_all();
      }
    }
  }

  int prepare(int q) {
    CgPrep& c = prep_[q];
    if (c.ready) return SKIPM_OK;
    skipm_lp_s* lp = lps_[idx_[q]];
    ColPass nrm[2], cls[2], qin;
    CgCloseArgs close;
    batch_cg_passes(lp, nrm, c.fin, cls, &qin, &c.init, &close);
    c.a_n.assign(2 * ab_, 0);
    c.a_c.assign(2 * ab_, 0);
    c.a_q.assign(ab_, 0);
    ColKey kk;
    for (int p = 0; p < 2; ++p) {
      c.nb_n = colpass_prepare(nrm[p], &c.a_n[p * ab_], &c.kn);
      c.nb_c = colpass_prepare(cls[p], &c.a_c[p * ab_], &kk);
      c.fin[p].nblk = c.nb_n;
    }
    c.nb_q = colpass_prepare(qin, &c.a_q[0], &c.kd);
    if (c.nb_n < 0 || c.nb_c < 0 || c.nb_q < 0 || !(kk == c.kd))
      return set_error("grouped CG: pass not covered"), SKIPM_EINVAL;
    c.fnb = finish_nblk(lp->m);
    c.is = lp->is;
    c.ready = true;
    return SKIPM_OK;
  }

  void* dp(size_t o) { return (void*)(dbuf_ + o); }

  // Work lists and arguments of the LPs `list` on the device (on cg_st_): the
  // CG set-up passes (init) or the three passes of an iteration with their
  // iteration offsets.  Callers have synchronised cg_st_ since its last use
  // of the staging buffers.
  int stage(const std::vector<int>& list, const std::vector<int64_t>* kstart, bool init) {
    const int na = (int)list.size();
    std::vector<ColKey> kn(na), kd(na);
    std::vector<int> bn(na), bc(na), bq(na);
    for (int q = 0; q < na; ++q) {
      const CgPrep& c = prep_[list[q]];
      kn[q] = c.kn;
      kd[q] = c.kd;
      bn[q] = c.nb_n;
      bc[q] = c.nb_c;
      bq[q] = c.nb_q;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
      off = (off + 255) / 256 * 256;
      const size_t o = off;
      off += bytes;
      return o;
    };
    std::vector<int64_t> kst_n, kst_d;
    if (init) {
      gq_ = group_by(kd, bq);
      for (auto& g : gq_) {
        g.args_off = take(g.members.size() * ab_);
        g.first_off = take(g.first.size() * sizeof(int32_t));
      }
      init_off_ = take(na * sizeof(CgInitArgs));
    } else {
      gn_ = group_by(kn, bn);
      gd_ = group_by(kd, bc);
      for (auto* G : {&gn_, &gd_})
        for (auto& g : *G) {
          g.args_off = take(2 * g.members.size() * ab_);
          g.first_off = take(g.first.size() * sizeof(int32_t));
          g.kst_off = take(g.members.size() * sizeof(int64_t));
        }
      ffirst_.assign(na + 1, 0);
      for (int q = 0; q < na; ++q) ffirst_[q + 1] = ffirst_[q] + prep_[list[q]].fnb;
      fin_off_ = take(2 * na * sizeof(FinishDotArgs));
      ffirst_off_ = take((na + 1) * sizeof(int32_t));
      kstart_off_ = take(na * sizeof(int64_t));
      isp_off_ = take(na * sizeof(int32_t*));
      flags_off_ = take(3 * na * sizeof(int32_t));
    }
    SK_TRY(reserve(off, 3 * na));
    auto put = [&](size_t o, const void* src, size_t bytes) { memcpy(hbuf_ + o, src, bytes); };
    if (init) {
      for (auto& g : gq_) {
        for (size_t q = 0; q < g.members.size(); ++q)
          put(g.args_off + q * ab_, prep_[list[g.members[q]]].a_q.data(), ab_);
        put(g.first_off, g.first.data(), g.first.size() * sizeof(int32_t));
      }
      for (int q = 0; q < na; ++q)
        put(init_off_ + q * sizeof(CgInitArgs), &prep_[list[q]].init, sizeof(CgInitArgs));
    } else {
      for (auto* G : {&gn_, &gd_})
        for (auto& g : *G) {
          const bool product = G == &gn_;
          for (size_t q = 0; q < g.members.size(); ++q) {
            const CgPrep& c = prep_[list[g.members[q]]];
            put(g.args_off + 2 * q * ab_, (product ? c.a_n : c.a_c).data(), 2 * ab_);
            const int64_t k0 = (*kstart)[g.members[q]];
            put(g.kst_off + q * sizeof(int64_t), &k0, sizeof(int64_t));
          }
          put(g.first_off, g.first.data(), g.first.size() * sizeof(int32_t));
        }
      for (int q = 0; q < na; ++q) {
        const CgPrep& c = prep_[list[q]];
        put(fin_off_ + 2 * q * sizeof(FinishDotArgs), c.fin, 2 * sizeof(FinishDotArgs));
        put(kstart_off_ + q * sizeof(int64_t), &(*kstart)[q], sizeof(int64_t));
        put(isp_off_ + q * sizeof(int32_t*), &c.is, sizeof(int32_t*));
      }
      put(ffirst_off_, ffirst_.data(), ffirst_.size() * sizeof(int32_t));
    }
    SK_CHECK_HIP(hipMemcpyAsync(dbuf_, hbuf_, off, hipMemcpyHostToDevice, cg_st_));
    return SKIPM_OK;
  }

  int reserve(size_t bytes, int nflags) {
    if (bytes > cap_) {
      SK_CHECK_HIP(hipStreamSynchronize(cg_st_));
      if (dbuf_) (void)hipFree(dbuf_);
      if (hbuf_) (void)hipHostFree(hbuf_);
      dbuf_ = nullptr;
      hbuf_ = nullptr;
      cap_ = 0;
      const size_t c = bytes + bytes / 2 + 4096;
      if (hipMalloc((void**)&dbuf_, c) != hipSuccess || hipHostMalloc((void**)&hbuf_, c) != hipSuccess)
        return set_error("grouped CG: staging allocation failed"), SKIPM_ENOMEM;
      cap_ = c;
    }
    if (nflags > nflags_cap_) {
      if (hflags_) (void)hipHostFree(hflags_);
      hflags_ = nullptr;
      if (hipHostMalloc((void**)&hflags_, nflags * sizeof(int32_t)) != hipSuccess)
        return set_error("grouped CG: flag buffer allocation failed"), SKIPM_ENOMEM;
      nflags_cap_ = nflags;
    }
    return SKIPM_OK;
  }

  skipm_lp_t* lps_;
  skipm_result* res_;
  std::vector<int> idx_;
  int nthreads_, dev_;
  std::vector<BatchLp> st_;
  std::vector<CgPrep> prep_;
  size_t ab_ = 0;
  hipStream_t cg_st_ = nullptr;
  std::vector<hipStream_t> streams_;
  // shared between the executor and the workers
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Task> tasks_;
  std::deque<int> ready_;
  int outstanding_ = 0;
  bool stop_ = false;
  int fatal_ = SKIPM_OK;
  std::string fatal_msg_;
  // staged work lists
  std::vector<Group> gn_, gd_, gq_;
  std::vector<int32_t> ffirst_;
  size_t fin_off_ = 0, ffirst_off_ = 0, kstart_off_ = 0, init_off_ = 0, isp_off_ = 0,
         flags_off_ = 0;
  char* dbuf_ = nullptr;
  char* hbuf_ = nullptr;
  size_t cap_ = 0;
  int32_t* hflags_ = nullptr;
  int nflags_cap_ = 0;
};

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
  // dense FP64-product LPs of this device go through the grouped engine; the
  // others (CSR, low-precision products) the single-LP way (threads below)
  std::vector<int> grouped_idx, single_idx;
  for (int i = 0; i < count; ++i) {
    skipm_lp_s* lp = lps[i];
    const bool g = lp->device == dev && batch_groupable(lp);
    (g ? grouped_idx : single_idx).push_back(i);
  }
  int grc = SKIPM_OK;
  std::string gerr;
  std::thread grouped_thread;
  if (!grouped_idx.empty()) {
    grouped_thread = std::thread([&] {
      Engine eng(lps, res, grouped_idx, std::max(1, std::min<int>(nw, (int)grouped_idx.size())),
                 dev);
      grc = eng.run(&gerr);
    });
  }
  const int nsingle = std::min<int>(nw, (int)single_idx.size());
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
      const int q = next.fetch_add(1);
      if (q >= (int)single_idx.size() || fatal.load() != SKIPM_OK) break;
      const int i = single_idx[q];
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
  pool.reserve(nsingle);
  for (int t = 0; t < nsingle; ++t) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  if (grouped_thread.joinable()) grouped_thread.join();
  if (fatal.load() != SKIPM_OK) {
    set_error(first_err.empty() ? "device error in batch" : first_err);
    return fatal.load();
  }
  if (grc != SKIPM_OK) {
    set_error(gerr.empty() ? "device error in batch" : gerr);
    return grc;
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
