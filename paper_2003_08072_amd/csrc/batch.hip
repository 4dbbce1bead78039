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
#include <functional>
#include <algorithm>
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
//     launches: per CG iteration one launch per pass (product pass, finish,
//     Q^{-1} pass) and block size / register class of the LPs' lane-group
//     shapes, whose work list is the (LP, workgroup) pairs of its LPs.  Every LP keeps the workgroup count,
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

// bytes of the copy of A that an LP's CG products read
int64_t cg_bytes(const skipm_lp_s* lp) {
  return lp->lda * lp->n * (lp->a_dtype == SKIPM_F64 ? 8 : 4);
}

// One LP in the engine: its handle and result, its loop state, its prepared
// CG arguments, and what to do when its run has ended (called on a worker
// thread, with that worker's stream, after the engine has let go of it).
struct Entry {
  skipm_lp_s* lp = nullptr;
  skipm_result* res = nullptr;
  BatchLp b;
  CgPrep prep;
  std::function<void(Entry*, hipStream_t)> done;
};

class Engine {
 public:
  Engine(int nthreads, int dev) : nthreads_(std::max(1, nthreads)), dev_(dev) {}
  ~Engine() {
    stop();
    if (dbuf_) (void)hipFree(dbuf_);
    if (hbuf_) (void)hipHostFree(hbuf_);
    if (hflags_) (void)hipHostFree(hflags_);
  }

  // Streams, worker threads and the executor thread.
  int start(std::string* err) {
    if (hipSetDevice(dev_) != hipSuccess) return *err = "hipSetDevice failed", SKIPM_EDEVICE;
    ab_ = colpass_args_bytes();
    bool ok = hipStreamCreateWithFlags(&cg_st_, hipStreamNonBlocking) == hipSuccess;
    if (hipEventCreateWithFlags(&cg_ev_, hipEventDisableTiming) != hipSuccess) cg_ev_ = nullptr;
    streams_.assign(nthreads_, nullptr);
    for (auto& st : streams_)
      ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
      *err = "could not create the engine's streams";
      destroy_streams();
      return SKIPM_EDEVICE;
    }
    for (int t = 0; t < nthreads_; ++t) pool_.emplace_back([this, t] { worker(t); });
    exec_ = std::thread([this] { executor(); });
    started_ = true;
    return SKIPM_OK;
  }

  // Queue an LP from its current iterate (thread-safe); e lives until e->done.
  // Returns the engine's fatal status instead (nothing queued) once an error
  // has stopped it.
  int add(Entry* e) {
    memset(e->res, 0, sizeof(*e->res));
    e->b = BatchLp{};
    std::lock_guard<std::mutex> g(mu_);
    if (fatal_ != SKIPM_OK) {
      e->res->status = fatal_;
      return fatal_;
    }
    ++outstanding_;
    live_.push_back(e);
    live_bytes_ += cg_bytes(e->lp);
    tasks_.push_back({e, false});
    cv_.notify_all();
    return SKIPM_OK;
  }

  // Wait for every queued LP, then end the threads.  After a fatal error the
  // LPs still in the engine end with that status.
  void stop() {
    if (!started_) return;
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    if (exec_.joinable()) exec_.join();
    for (auto& th : pool_) th.join();
    pool_.clear();
    std::vector<Entry*> left;
    {
      std::lock_guard<std::mutex> g(mu_);
      left.swap(live_);
      live_bytes_ = 0;
      outstanding_ = 0;
    }
    for (Entry* e : left) {
      e->res->status = fatal_;
      e->b.rc = fatal_;
      e->b.active = false;
      if (e->done) e->done(e, cg_st_);
    }
    destroy_streams();
    started_ = false;
  }

  int fatal(std::string* msg) {
    std::lock_guard<std::mutex> g(mu_);
    if (msg) *msg = fatal_msg_;
    return fatal_;
  }

 private:
  struct Task {
    Entry* e;
    bool after_cg;  // run the end of the iteration first
  };

  void destroy_streams() {
    for (auto& st : streams_)
      if (st) (void)hipStreamDestroy(st);
    streams_.clear();
    if (cg_st_) (void)hipStreamDestroy(cg_st_);
    cg_st_ = nullptr;
    if (cg_ev_) (void)hipEventDestroy(cg_ev_);
    cg_ev_ = nullptr;
  }

  void set_fatal(int rc, const std::string& msg) {
    if (fatal_ == SKIPM_OK) {
      fatal_ = rc;
      fatal_msg_ = msg;
    }
  }

  // Called by each engine thread as it ends.  After an error the threads end
  // with LPs still queued or in the CG; the last thread out (no other thread
  // can then hold an LP) ends those LPs with the error, so that their owners
  // (a waiting request of the server) learn of it instead of waiting on.
  void thread_exit(hipStream_t s) {
    std::vector<Entry*> left;
    int rc = SKIPM_OK;
    {
      std::lock_guard<std::mutex> g(mu_);
      if (++exited_ < nthreads_ + 1 || fatal_ == SKIPM_OK) return;
      rc = fatal_;
      left.swap(live_);
      live_bytes_ = 0;
      tasks_.clear();
      ready_.clear();
      outstanding_ = 0;
    }
    for (Entry* e : left) {
      e->res->status = rc;
      e->b.rc = rc;
      e->b.active = false;
      if (e->done) e->done(e, s);
    }
  }

  void worker(int t) {
    (void)hipSetDevice(dev_);
    hipStream_t s = streams_[t];
    // the end of each phase is awaited by polling this event (a plain stream
    // synchronisation if it cannot be made)
    hipEvent_t wev = nullptr;
    if (hipEventCreateWithFlags(&wev, hipEventDisableTiming) != hipSuccess) wev = nullptr;
    for (;;) {
      Task task;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] {
          return fatal_ != SKIPM_OK || !tasks_.empty() || (stop_ && outstanding_ == 0);
        });
        if (fatal_ != SKIPM_OK || tasks_.empty()) break;
        task = tasks_.front();
        tasks_.pop_front();
      }
      Entry* e = task.e;
      if (task.after_cg) {
        batch_phase_b(e->lp, e->res, &e->b, s);
        (void)wait_stream(s, wev);
      }
      if (e->b.active) {
        batch_phase_a(e->lp, e->res, &e->b, s);
        (void)wait_stream(s, wev);
      }
      bool finished = false;
      {
        std::lock_guard<std::mutex> g(mu_);
        if (e->b.rc != SKIPM_OK) set_fatal(e->b.rc, e->b.err);
        if (!e->b.active) {
          finished = true;
          live_.erase(std::find(live_.begin(), live_.end(), e));
          live_bytes_ -= cg_bytes(e->lp);
        } else if (e->b.grouped) {
          ready_.push_back(e);
        } else {
          tasks_.push_back({e, true});  // its CG ran in one workgroup
        }
      }
      if (finished && e->done) e->done(e, s);
      if (finished) {
        std::lock_guard<std::mutex> g(mu_);
        --outstanding_;
      }
      cv_.notify_all();
    }
    if (wev) (void)hipEventDestroy(wev);
    thread_exit(s);
  }

  // The executor: the grouped CG of the LPs that are ready, chunk by chunk.
  void executor() {
    (void)hipSetDevice(dev_);
    std::vector<Entry*> in_cg;    // LPs in the grouped CG
    std::vector<int64_t> kstart;  // their next CG iteration
    for (;;) {
      std::vector<Entry*> fresh;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (in_cg.empty())
          cv_.wait(lk, [&] {
            return !ready_.empty() || fatal_ != SKIPM_OK || (stop_ && outstanding_ == 0);
          });
        if (fatal_ != SKIPM_OK) break;
        if (in_cg.empty() && ready_.empty()) {
          if (stop_ && outstanding_ == 0) break;
          continue;
        }
        fresh.assign(ready_.begin(), ready_.end());
        ready_.clear();
      }
      const int rc = step(fresh, &in_cg, &kstart);
      if (rc != SKIPM_OK) {
        std::lock_guard<std::mutex> g(mu_);
        set_fatal(rc, skipm_last_error());
        cv_.notify_all();
        break;
      }
    }
    // an error leaves this thread's LPs with the last thread out
    (void)hipStreamSynchronize(cg_st_);
    thread_exit(cg_st_);
  }

  // Set up the newcomers' CG, then one chunk of grouped iterations for all
  // LPs in the CG; those done go back to the workers.
  int step(const std::vector<Entry*>& fresh, std::vector<Entry*>* in_cg,
           std::vector<int64_t>* kstart) {
    if (!fresh.empty()) {
      for (Entry* e : fresh) SK_TRY(prepare(e));
      // z_0 = Q^{-1} p, then r, z, d, x and the stopping threshold
      SK_TRY(stage(fresh, nullptr, true));
      for (auto& g : gq_)
        if (launch_colpass_grouped(g.key, dp(g.args_off), (const int32_t*)dp(g.first_off),
                                   (int)g.members.size(), g.first.back(), nullptr, 0, cg_st_) != 0)
          return set_error("grouped CG: no kernel for a shape"), SKIPM_EINVAL;
      launch_cg_init_grouped((const CgInitArgs*)dp(init_off_), (int)fresh.size(), cg_st_);
      SK_CHECK_HIP(hipGetLastError());
      for (Entry* e : fresh) {
        in_cg->push_back(e);
        kstart->push_back(0);
      }
      SK_CHECK_HIP(hipStreamSynchronize(cg_st_));  // the staging buffer is reused below
    }
    if (in_cg->empty()) return SKIPM_OK;
    SK_TRY(stage(*in_cg, kstart, false));
    const int na = (int)in_cg->size();
    const int64_t* ks = (const int64_t*)dp(kstart_off_);
    for (int j = 0; j < kChunk; ++j) {
      for (auto* G : {&gn_, &gd_}) {
        if (G == &gd_)
          launch_finish_dot_grouped((const FinishDotArgs*)dp(fin_off_),
                                    (const int32_t*)dp(ffirst_off_), na, ffirst_.back(), ks, j,
                                    cg_st_);
        for (auto& g : *G)
          if (launch_colpass_grouped(g.key, dp(g.args_off), (const int32_t*)dp(g.first_off),
                                     (int)g.members.size(), g.first.back(),
                                     (const int64_t*)dp(g.kst_off), j, cg_st_) != 0)
            return set_error("grouped CG: no kernel for a shape"), SKIPM_EINVAL;
      }
    }
    launch_cg_flags((int32_t* const*)dp(isp_off_), na, (int32_t*)dp(flags_off_), cg_st_);
    SK_CHECK_HIP(hipGetLastError());
    SK_CHECK_HIP(hipMemcpyAsync(hflags_, dp(flags_off_), 3 * na * sizeof(int32_t),
                                hipMemcpyDeviceToHost, cg_st_));
    SK_TRY(wait_stream(cg_st_, cg_ev_));
    std::vector<Entry*> keep, finished;
    std::vector<int64_t> kkeep;
    for (int q = 0; q < na; ++q) {
      Entry* e = (*in_cg)[q];
      if (hflags_[3 * q]) {
        e->b.its = hflags_[3 * q + 1];
        e->b.fail = hflags_[3 * q + 2] ? 1 : 0;
        finished.push_back(e);
      } else {
        keep.push_back(e);
        kkeep.push_back((*kstart)[q] + kChunk);
      }
    }
    in_cg->swap(keep);
    kstart->swap(kkeep);
    if (!finished.empty()) {
      std::lock_guard<std::mutex> g(mu_);
      for (Entry* e : finished) tasks_.push_back({e, true});
      cv_.notify_all();
    }
    return SKIPM_OK;
  }

  int prepare(Entry* e) {
    CgPrep& c = e->prep;
    if (c.ready) return SKIPM_OK;
    ColPass nrm[2], cls[2], qin;
    CgCloseArgs close;
    batch_cg_passes(e->lp, nrm, c.fin, cls, &qin, &c.init, &close);
    {
      // the grouped products of all LPs in the engine stream more than the
      // Infinity Cache holds: non-temporal loads (the same sums)
      std::lock_guard<std::mutex> g(mu_);
      if (live_bytes_ > kStreamBytes) nrm[0].nt = nrm[1].nt = 1;
    }
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
    c.fnb = finish_nblk(e->lp->m);
    c.is = e->lp->is;
    c.ready = true;
    return SKIPM_OK;
  }

  void* dp(size_t o) { return (void*)(dbuf_ + o); }

  // Work lists and arguments of the LPs `list` on the device (on cg_st_): the
  // CG set-up pass (init) or the three passes of an iteration with each LP's
  // iteration offset.  Callers have synchronised cg_st_ since its last use of
  // the staging buffers.
  int stage(const std::vector<Entry*>& list, const std::vector<int64_t>* kstart, bool init) {
    const int na = (int)list.size();
    std::vector<ColKey> kn(na), kd(na);
    std::vector<int> bn(na), bc(na), bq(na);
    for (int q = 0; q < na; ++q) {
      const CgPrep& c = list[q]->prep;
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
      for (int q = 0; q < na; ++q) ffirst_[q + 1] = ffirst_[q] + list[q]->prep.fnb;
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
          put(g.args_off + q * ab_, list[g.members[q]]->prep.a_q.data(), ab_);
        put(g.first_off, g.first.data(), g.first.size() * sizeof(int32_t));
      }
      for (int q = 0; q < na; ++q)
        put(init_off_ + q * sizeof(CgInitArgs), &list[q]->prep.init, sizeof(CgInitArgs));
    } else {
      for (auto* G : {&gn_, &gd_})
        for (auto& g : *G) {
          const bool product = G == &gn_;
          for (size_t q = 0; q < g.members.size(); ++q) {
            const CgPrep& c = list[g.members[q]]->prep;
            put(g.args_off + 2 * q * ab_, (product ? c.a_n : c.a_c).data(), 2 * ab_);
            const int64_t k0 = (*kstart)[g.members[q]];
            put(g.kst_off + q * sizeof(int64_t), &k0, sizeof(int64_t));
          }
          put(g.first_off, g.first.data(), g.first.size() * sizeof(int32_t));
        }
      for (int q = 0; q < na; ++q) {
        const CgPrep& c = list[q]->prep;
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

  int nthreads_, dev_;
  bool started_ = false;
  size_t ab_ = 0;
  hipStream_t cg_st_ = nullptr;
  hipEvent_t cg_ev_ = nullptr;  // the end of each chunk, awaited by polling
  std::vector<hipStream_t> streams_;
  std::vector<std::thread> pool_;
  std::thread exec_;
  // shared between the executor, the workers and add()
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Task> tasks_;
  std::deque<Entry*> ready_;
  std::vector<Entry*> live_;
  int64_t live_bytes_ = 0;  // bytes of the CG copies of A of the LPs in live_
  int outstanding_ = 0;
  int exited_ = 0;  // engine threads that have ended
  bool stop_ = false;
  int fatal_ = SKIPM_OK;
  std::string fatal_msg_;
  // staged work lists (executor only)
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
  // several LPs share the device: CG chunks are checked with their stream idle
  // (the flag is restored on return)
  std::vector<char> overlap(count);
  for (int i = 0; i < count; ++i) {
    overlap[i] = lps[i]->overlap_checks;
    lps[i]->overlap_checks = false;
  }
  struct Restore {
    skipm_lp_t* lps;
    const std::vector<char>& v;
    ~Restore() {
      for (size_t i = 0; i < v.size(); ++i) lps[i]->overlap_checks = v[i] != 0;
    }
  } restore{lps, overlap};
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
      Engine eng(std::min<int>(nw, (int)grouped_idx.size()), dev);
      grc = eng.start(&gerr);
      if (grc != SKIPM_OK) return;
      std::vector<Entry> entries(grouped_idx.size());
      for (size_t q = 0; q < grouped_idx.size(); ++q) {
        entries[q].lp = lps[grouped_idx[q]];
        entries[q].res = &res[grouped_idx[q]];
        eng.add(&entries[q]);
      }
      eng.stop();  // waits for every LP
      grc = eng.fatal(&gerr);
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
    skipm_result res{};          // filled by the engine while the request runs
    Entry entry;                 // the request's place in the grouped engine
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
  Engine* engine = nullptr;          // the grouped CG of the dense requests in flight
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
  void worker_main();
  void finish(Req* r, skipm_lp_t lp, const Outcome& oc0, hipStream_t st);
};

// The end of a request: copy x out, count the device bytes, free the LP, then
// publish the outcome into r->info under the lock (srv_poll never sees a
// half-written result) and release its slot and footprint.
void skipm_server_s::finish(Req* r, skipm_lp_t lp, const Outcome& oc0, hipStream_t st) {
  Outcome oc = oc0;
  if (lp) {
    if (oc.rc == SKIPM_OK && r->x_out) oc.rc = lp_get_iterate(lp, r->x_out, nullptr, nullptr, st);
    int64_t held = 0;
    lp_device_bytes(lp, &held);
    oc.device_bytes = held;
    lp_destroy(lp);
  }
  {
    std::lock_guard<std::mutex> g(mu);
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
  }
  work_cv.notify_all();
  done_cv.notify_all();
}

// A slot: admit the request at the head of the queue once it fits, create its
// LP; a dense LP with FP64 CG products joins the grouped engine (and the slot
// is free for the next admission at once), any other is solved here.
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
    skipm_lp_t lp = nullptr;
    int rc = have_stream ? SKIPM_OK : SKIPM_EDEVICE;
    if (rc == SKIPM_OK && r->ready && hipStreamWaitEvent(st, r->ready, 0) != hipSuccess)
      rc = SKIPM_EDEVICE;
    if (rc == SKIPM_OK) rc = lp_create(&lp, &r->prob, &r->prm, st);
    if (rc == SKIPM_OK) lp->overlap_checks = false;  // other requests share the device
    if (rc != SKIPM_OK) {
      oc.rc = rc;
      oc.res.status = rc;
      finish(r, nullptr, oc, st);
      continue;
    }
    if (engine && batch_groupable(lp)) {
      r->entry.lp = lp;
      r->entry.res = &r->res;
      r->entry.done = [this, r](Entry* e, hipStream_t s) {
        Outcome o;
        o.res = *e->res;
        o.rc = e->b.rc;
        finish(r, e->lp, o, s);
      };
      if (engine->add(&r->entry) == SKIPM_OK) continue;
      // the engine stopped on an error: this request (its LP untouched) is
      // solved on the slot
    }
    rc = lp_solve(lp, &oc.res, st);
    if (rc == SKIPM_ENOTCONV || rc == SKIPM_ESTALL || rc == SKIPM_ERANK || rc == SKIPM_ENAN)
      rc = SKIPM_OK;  // an outcome of the LP, in res.status
    oc.rc = rc;
    finish(r, lp, oc, st);
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
  s->engine = new Engine(std::min(slots, 16), s->device);
  std::string err;
  if (s->engine->start(&err) != SKIPM_OK) {
    delete s->engine;
    delete s;
    return set_error(err), SKIPM_EDEVICE;
  }
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
  if (srv->engine) {
    srv->engine->stop();  // the dense requests still in the grouped engine
    delete srv->engine;
    srv->engine = nullptr;
  }
  for (auto& kv : srv->reqs) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  delete srv;
  return SKIPM_OK;
}

}  // extern "C"
