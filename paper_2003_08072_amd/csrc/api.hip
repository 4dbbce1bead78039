// C ABI of libskipm and the host-side control of the IPM (Alg. 2 with Alg. 1 inside).
//
// One IPM iteration, all on the handle's stream:
//   prologue pass over A  -> r_d, d^2, r_p, p (eq. pdef), ||r||, c^T x, b^T y
//   [host reads ~10 scalars: stopping test]
//   hash + bucket sort     -> W of step (a)
//   sketch pass over A     -> B = A D W (Alg. 1 step 1)
//   Gram + Cholesky        -> Q^{-1} = (B B^T)^{-1} = L^{-T} L^{-1}
//   CG, per iteration: normal pass over A (one read; it also takes the stop
//       test, beta and d_k), partial sums with d^T q, and the Q^{-1} pass that
//       takes alpha and updates x, r, z; chunks of iterations are enqueued and
//       the host reads the done flag once per chunk (dense FP64 LPs with
//       m <= 64: the whole CG in one workgroup)
//   epilogue pass over A   -> ds (eq. delshat), g = A D^2 A^T dy - p
//   t = (A D W)^+ g by refinement on the true residual g - B t (FP64)
//   direction pass         -> v (eq. compv), dx (eq. delxhat), step sums
//   step pass + finalize   -> alpha_max, alpha (Alg. 2 steps e, f)
//   update pass            -> (x, y, s) (step g), mu
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "common.h"
#include "handle.h"
#include "vrefine.h"

namespace skipm {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace skipm

using namespace skipm;

namespace {

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

template <typename T>
int dalloc(skipm_lp_s* lp, T** out, int64_t count) {
  void* p = nullptr;
  const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return SKIPM_ENOMEM;
  }
  lp->allocs.push_back(p);
  lp->bytes += (int64_t)bytes;
  *out = (T*)p;
  return SKIPM_OK;
}

int validate_params(const skipm_params& p, int64_t m, int64_t n) {
  if (!(p.sigma > 0.0 && p.sigma < 0.8)) return set_error("sigma must lie in (0, 0.8)"), SKIPM_EINVAL;
  if (!(p.gamma > 0.0 && p.gamma < 1.0)) return set_error("gamma must lie in (0, 1)"), SKIPM_EINVAL;
  if (!(p.guard >= 0.0 && p.guard < 1.0)) return set_error("guard must lie in [0, 1)"), SKIPM_EINVAL;
  const int64_t w = p.w > 0 ? p.w : 4 * m;
  if (w < m) return set_error("sketch width w must be >= m"), SKIPM_EINVAL;
  if (p.s < 1 || p.s > 16) return set_error("s must lie in [1, 16]"), SKIPM_EINVAL;
  if (w % p.s != 0) return set_error("s must divide w"), SKIPM_EINVAL;
  if (p.max_cg < 1 || p.max_outer < 0) return set_error("bad iteration caps"), SKIPM_EINVAL;
  if (p.precision != SKIPM_PREC_FP64 && p.precision != SKIPM_PREC_MIXED &&
      p.precision != SKIPM_PREC_BF16)
    return set_error("unknown precision"), SKIPM_EINVAL;
  if (p.inner != SKIPM_INNER_CG && p.inner != SKIPM_INNER_SD && p.inner != SKIPM_INNER_RICHARDSON)
    return set_error("unknown inner solver"), SKIPM_EINVAL;
  if (p.sketch != SKIPM_SKETCH_COUNT && p.sketch != SKIPM_SKETCH_GAUSSIAN)
    return set_error("unknown sketch"), SKIPM_EINVAL;
  if (n * p.s > INT32_MAX) return set_error("n*s exceeds int32 item indices"), SKIPM_EINVAL;
  return SKIPM_OK;
}

constexpr size_t kScalarBlockBytes = S_NSLOTS * sizeof(double) + I_NINTS * sizeof(int32_t);

int sync_read(skipm_lp_s* lp, hipStream_t st) {
  SK_CHECK_HIP(hipMemcpyAsync(lp->hsc, lp->sc, kScalarBlockBytes, hipMemcpyDeviceToHost, st));
  return wait_stream(st, lp->rd_ev);
}

const int32_t* host_ints(const skipm_lp_s* lp) { return (const int32_t*)(lp->hsc + S_NSLOTS); }

}  // namespace

namespace skipm {

// The host's waits on the device (reads of the scalar block, CG checks, the
// batch's phase ends) sit between short chains of dependent launches: the GPU
// idles from the awaited work's end until the host has woken up and queued
// the next launch.  So the host polls the event for a while (at most
// kSpinUs) before a blocking wait (config 0: 45.3 -> 50.3 solves/s).
constexpr int kSpinUs = 200;

int poll_event(hipEvent_t ev) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) return SKIPM_OK;
    if (e != hipErrorNotReady) {
      set_error(std::string("hipEventQuery: ") + hipGetErrorString(e));
      return SKIPM_EDEVICE;
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinUs)) break;
  }
  SK_CHECK_HIP(hipEventSynchronize(ev));
  return SKIPM_OK;
}

int wait_stream(hipStream_t st, hipEvent_t ev) {
  if (!ev) {
    SK_CHECK_HIP(hipStreamSynchronize(st));
    return SKIPM_OK;
  }
  SK_CHECK_HIP(hipEventRecord(ev, st));
  return poll_event(ev);
}

}  // namespace skipm

namespace {

int mu_from_iterate(skipm_lp_s* lp, hipStream_t st) {
  launch_xs_sum(lp->n, lp->x, lp->sv, lp->red, lp->nblk_vec, st);
  launch_mu_finalize(lp->red, lp->nblk_vec, lp->n, lp->sc, st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

int set_param_slots(skipm_lp_s* lp, hipStream_t st) {
  double vals[3] = {lp->prm.sigma, lp->prm.gamma, lp->prm.guard};
  SK_CHECK_HIP(hipMemcpyAsync(lp->sc + S_SIGMA, vals, sizeof(vals), hipMemcpyHostToDevice, st));
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

// ---- passes ----------------------------------------------------------------

int run_colpass(ColPass& cp, hipStream_t st) {
  if (launch_colpass(cp, st) != 0) {
    set_error("no column-pass kernel for this shape / type");
    return SKIPM_EINVAL;
  }
  return SKIPM_OK;
}

int stream_A(const skipm_lp_s* lp, int ta) {
  const int64_t bytes = ta == SKIPM_F64 ? lp->lda * lp->n * 8
                        : ta == SKIPM_F32 ? lp->lda * lp->n * 4
                                          : lp->lda16 * lp->n * 2;
  return bytes > kStreamBytes ? 1 : 0;
}

// The CG products read the copy of A of the current precision tier: FP32 or
// BF16 values, widened and accumulated in FP64.
void use_tier_copy(skipm_lp_s* lp, ColPass& cp) {
  if (lp->tier == SKIPM_TIER_FP32) {
    cp.A = lp->A32;
    cp.ta = SKIPM_F32;
    cp.nt = stream_A(lp, SKIPM_F32);
    cp.nblk = lp->nblk_A32;
  } else if (lp->tier == SKIPM_TIER_BF16) {
    cp.A = lp->A16;
    cp.ta = kTypeBF16;
    cp.lda = lp->lda16;
    cp.nt = stream_A(lp, kTypeBF16);
    cp.nblk = lp->nblk_A16;
  }
}

ColPass colpass_A(skipm_lp_s* lp, int mode) {
  ColPass cp{};
  cp.nt = stream_A(lp, lp->a_dtype);
  cp.mode = mode;
  cp.A = lp->A;
  cp.ta = lp->a_dtype;
  cp.tc = SKIPM_F64;
  cp.lda = lp->lda;
  cp.m = lp->m;
  cp.n = lp->n;
  cp.part = lp->part;
  cp.ldp = lp->mp;
  cp.red = lp->red;
  cp.sc = lp->sc;
  cp.nblk = mode == COL_PROLOGUE ? lp->nblk_Ap : lp->nblk_A;
  return cp;
}

int prologue_sparse(skipm_lp_s* lp, hipStream_t st) {
  const SparseA& A = lp->sp;
  if (launch_csc_dot(A, COL_PROLOGUE, lp->y, lp->x, lp->sv, lp->c, nullptr, nullptr, nullptr,
                     lp->cf2, lp->rd, lp->d2, nullptr, lp->red, lp->sc, nullptr, lp->nblk_csc,
                     st) != 0)
    return set_error("m too large for the sparse path"), SKIPM_EINVAL;
  // r_p = A x - b ; p = b - A (sigma mu / s + d2 r_d)
  launch_csr_segsum(A, lp->x, lp->cf2, lp->segsum, nullptr, st);
  launch_csr_fold(A, lp->segsum, 0, 1.0, lp->b, -1.0, lp->rp, nullptr, st);
  launch_csr_fold(A, lp->segsum, 1, -1.0, lp->b, 1.0, lp->p, nullptr, st);
  launch_prologue_finalize(lp->m, lp->rp, lp->b, lp->y, lp->red, lp->nblk_csc, lp->sc,
                           lp->origin_pending, st);
  lp->origin_pending = 0;
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

// out = scale * A D^2 A^T u + beta * add, sparse A (two passes + fold)
int normal_sparse(skipm_lp_s* lp, const double* u, double scale, const double* add, double beta,
                  double* out, const int32_t* done, hipStream_t st) {
  const SparseA& A = lp->sp;
  if (launch_sb_normal(A, u, lp->d2, lp->part, lp->mp, done, st) != 0)
    return set_error("m too large for the sparse path"), SKIPM_EINVAL;
  launch_finish(lp->part, lp->mp, 0, (int)A.nbk, lp->m, scale, add, beta, out, done, st);
  return SKIPM_OK;
}

int prologue(skipm_lp_s* lp, hipStream_t st) {
  if (lp->fmt == SKIPM_CSR) return prologue_sparse(lp, st);
  ColPass cp = colpass_A(lp, COL_PROLOGUE);
  cp.u = lp->y;
  cp.x = lp->x;
  cp.s = lp->sv;
  cp.c = lp->c;
  cp.rd_out = lp->rd;
  cp.d2_out = lp->d2;
  SK_TRY(run_colpass(cp, st));
  // r_p = A x - b ; p = b - A (sigma mu / s + d2 r_d)
  launch_finish2(lp->part, 2 * lp->mp, cp.nblk, lp->m, 0, 1.0, lp->b, -1.0, lp->rp, lp->mp, -1.0,
                 lp->b, 1.0, lp->p, st);
  launch_prologue_finalize(lp->m, lp->rp, lp->b, lp->y, lp->red, cp.nblk, lp->sc,
                           lp->origin_pending, st);
  lp->origin_pending = 0;
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

int hash_items(skipm_lp_s* lp, int64_t salt, hipStream_t st) {
  if (lp->hashed_k == salt) return SKIPM_OK;
  launch_fill_i32(lp->bcnt, 0, lp->w, st);
  launch_hash(lp->prm.seed, salt, lp->s, lp->n, lp->w, lp->bucket, lp->sign, lp->bcnt, st);
  launch_bucket_scan(lp->bcnt, lp->bptr, lp->bcur, lp->w, st);
  launch_bucket_scatter(lp->bucket, lp->n * lp->s, lp->w, lp->bptr, lp->bcur, lp->perm_raw, st);
  launch_bucket_sort(lp->bptr, lp->perm_raw, lp->perm, lp->w, st);
  SK_CHECK_HIP(hipGetLastError());
  lp->hashed_k = salt;
  return SKIPM_OK;
}

int factor(skipm_lp_s* lp, double shift, hipStream_t st) {
  launch_gram(lp->B, lp->lda, lp->m, lp->w, lp->Gpart, lp->ksplit, lp->mp, st);
  launch_gram_finish(lp->Gpart, lp->ksplit, lp->m, lp->mp, lp->G, st);
  if (shift > 0) launch_shift_diag(lp->G, lp->mp, lp->m, shift, st);
  // X = 0 (blocks above the diagonal stay zero) and the failure flag cleared
  launch_fill_f64_flag(lp->Xb, 0.0, lp->mp * lp->mp, lp->is + I_FACT_FAIL, st);
  launch_spd_inverse(lp->G, lp->Xb, lp->Ct, lp->mp, lp->is + I_FACT_FAIL, st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

// out = Q^{-1} u (u, out: m-vectors, padded to mp with zeros)
int qinv_apply(skipm_lp_s* lp, const double* u, double* out, const int32_t* done,
               hipStream_t st) {
  ColPass cp{};
  cp.mode = COL_DOT;
  cp.A = lp->G;
  cp.ta = SKIPM_F64;
  cp.tc = SKIPM_F64;
  cp.lda = lp->mp;
  cp.m = lp->mp;
  cp.n = lp->m;
  cp.u = u;
  cp.t_out = out;
  cp.done = done;
  cp.nblk = 0;
  return run_colpass(cp, st);
}

constexpr int kKtPairs = 64;
static_assert(kKtPairs <= 64, "one bit per event pair in kt_used");

// Takes an event pair for a timing sample of the product of CG iteration
// `iter` when sampling is on; returns the pair index or -1.
// Timing-only events: no system-scope fence (cache write-back and invalidate)
// when they are recorded, so they do not add that cost to the interval they
// bracket.  Results are never read through them (the stream is synchronised).
constexpr unsigned kTimingEvent = hipEventDisableSystemFence;

int kt_take(skipm_lp_s* lp, int iter) {
  if (lp->kt_every <= 0 || iter % lp->kt_every != 0) return -1;
  if (lp->kt_used == ~0ull) return -1;
  const int q = __builtin_ctzll(~lp->kt_used);
  lp->kt_used |= 1ull << q;
  lp->kt_iter.push_back(iter);
  lp->kt_tier.push_back(lp->fmt == SKIPM_CSR ? SKIPM_TIER_FP64 : lp->tier);
  lp->kt_pair.push_back(q);
  return q;
}

void kt_drop_last(skipm_lp_s* lp) {
  lp->kt_used &= ~(1ull << lp->kt_pair.back());
  lp->kt_iter.pop_back();
  lp->kt_tier.pop_back();
  lp->kt_pair.pop_back();
}

// Sparse product (three kernels): events recorded on the stream around them.
int kt_begin(skipm_lp_s* lp, int iter, hipStream_t st) {
  const int q = kt_take(lp, iter);
  if (q >= 0 && hipEventRecord(lp->kt_ev[2 * q], st) != hipSuccess) {
    kt_drop_last(lp);
    return -1;
  }
  return q;
}

void kt_end(skipm_lp_s* lp, int q, hipStream_t st) {
  if (q >= 0) (void)hipEventRecord(lp->kt_ev[2 * q + 1], st);  // a failed stamp drops the sample
}

// At a CG check: `executed` CG iterations have run by the snapshot the host
// read.  Samples of earlier iterations are taken; later ones stay pending
// (their products may still be queued) unless the CG is over (`final`), when
// they were skipped by the done flag and are dropped.
void kt_harvest(skipm_lp_s* lp, int executed, bool final) {
  size_t keep = 0;
  for (size_t q = 0; q < lp->kt_iter.size(); ++q) {
    const int pair = lp->kt_pair[q];
    if (lp->kt_iter[q] >= executed && !final) {
      lp->kt_iter[keep] = lp->kt_iter[q];
      lp->kt_tier[keep] = lp->kt_tier[q];
      lp->kt_pair[keep] = pair;
      ++keep;
      continue;
    }
    float ms = 0;
    if (lp->kt_iter[q] < executed &&
        hipEventElapsedTime(&ms, lp->kt_ev[2 * pair], lp->kt_ev[2 * pair + 1]) == hipSuccess) {
      lp->kt_sum_ms += ms;
      ++lp->kt_count;
      lp->kt_tier_ms[lp->kt_tier[q]] += ms;
      ++lp->kt_tier_n[lp->kt_tier[q]];
    }
    lp->kt_used &= ~(1ull << pair);
  }
  lp->kt_iter.resize(keep);
  lp->kt_tier.resize(keep);
  lp->kt_pair.resize(keep);
}

// The passes of a fused dense CG iteration of parity p (d_k lives in cd for
// even k, cd2 for odd k): the product pass that opens it, the finish that
// forms q and the d^T q partials, and the Q^{-1} pass that closes it.  cg.k is
// the caller's (the iteration).  The lone CG and the grouped batch CG launch
// exactly these arguments.
ColPass cg_normal_args(skipm_lp_s* lp, int p) {
  ColPass cp = colpass_A(lp, COL_NORMAL);
  cp.u = lp->cd;  // d_0 (written by the CG init) for iteration 0
  cp.d2 = lp->d2;
  use_tier_copy(lp, cp);
  cp.done = lp->is + I_CG_DONE;
  cp.cg.on = 1;
  cp.cg.inner = lp->prm.inner;
  cp.cg.z = lp->cz;
  cp.cg.d_old = p ? lp->cd : lp->cd2;
  cp.cg.d_new = p ? lp->cd2 : lp->cd;
  cp.cg.prz = lp->cgred + lp->cg_nf;
  cp.cg.np = lp->cg_nd;
  cp.cg.sc = lp->sc;
  cp.cg.is = lp->is;
  return cp;
}

FinishDotArgs cg_finish_args(skipm_lp_s* lp, int p, int nblk_product) {
  FinishDotArgs f;
  f.part = lp->part;
  f.ldp = lp->mp;
  f.nblk = nblk_product;
  f.m = lp->m;
  f.dvec = p ? lp->cd2 : lp->cd;
  f.out = lp->cq;
  f.dq_out = lp->cgred;
  f.done = lp->is + I_CG_DONE;
  return f;
}

ColPass cg_close_args(skipm_lp_s* lp, double* xsol, int p) {
  ColPass pq{};
  pq.mode = COL_DOT;
  pq.A = lp->G;
  pq.ta = SKIPM_F64;
  pq.tc = SKIPM_F64;
  pq.lda = lp->mp;
  pq.m = lp->mp;
  pq.n = lp->m;
  pq.u = lp->cq;
  pq.done = lp->is + I_CG_DONE;
  pq.nblk = lp->cg_nd;
  pq.cg.on = 1;
  pq.cg.inner = lp->prm.inner;
  pq.cg.sc = lp->sc;
  pq.cg.is = lp->is;
  pq.cg.q = lp->cq;
  pq.cg.d = p ? lp->cd2 : lp->cd;
  pq.cg.x = xsol;
  pq.cg.r = lp->cr;
  pq.cg.zz = lp->cz;
  pq.cg.pdq = lp->cgred;
  pq.cg.nf = lp->cg_nf;
  pq.cg.prz_out = lp->cgred + lp->cg_nf;
  pq.nt = lp->fmt == SKIPM_CSR;
  return pq;
}

// One CG iteration on A D^2 A^T (the chunk loop checks the done flag).
int pcg_iteration(skipm_lp_s* lp, double* xsol, int iter, hipStream_t st) {
  const int32_t* done = lp->is + I_CG_DONE;
  double* dk = (iter & 1) ? lp->cd2 : lp->cd;
  const double* dprev = (iter & 1) ? lp->cd : lp->cd2;
  double* pdq = lp->cgred;
  double* prz = lp->cgred + lp->cg_nf;
  if (lp->fmt == SKIPM_CSR) {
    // four launches per iteration: the column pass opens the iteration (stop
    // test, beta, d_k), the row pass and fold give q and d^T q partials, the
    // Q^{-1} pass closes it
    CgFuse cg{};
    cg.on = 1;
    cg.inner = lp->prm.inner;
    cg.k = iter;
    cg.z = lp->cz;
    cg.d_old = dprev;
    cg.d_new = dk;
    cg.prz = prz;
    cg.np = lp->cg_nd;
    cg.sc = lp->sc;
    cg.is = lp->is;
    const SparseA& A = lp->sp;
    const int q = kt_begin(lp, iter, st);
    if (launch_sb_normal(A, lp->cd, lp->d2, lp->part, lp->mp, done, st, &cg) != 0)
      return set_error("m too large for the sparse path"), SKIPM_EINVAL;
    if (launch_finish_dot(lp->part, lp->mp, (int)A.nbk, lp->m, dk, lp->cq, pdq, done, st) !=
        lp->cg_nf)
      return set_error("sparse CG: finish shape mismatch"), SKIPM_EINVAL;
    kt_end(lp, q, st);
  } else {
    // Three launches per iteration: the product pass opens the iteration (stop
    // test, beta, d_k), the finish adds d^T q partials, the Q^{-1} pass closes
    // it (alpha, x, r, z and r^T z partials).  d alternates between two buffers.
    ColPass cp = cg_normal_args(lp, iter & 1);
    cp.cg.k = iter;
    const int q = kt_take(lp, iter);
    if (q >= 0) {  // dense product: the runtime stamps the events with the kernel itself
      cp.ev0 = lp->kt_ev[2 * q];
      cp.ev1 = lp->kt_ev[2 * q + 1];
    }
    SK_TRY(run_colpass(cp, st));
    if (launch_finish_dot(lp->part, lp->mp, cp.nblk, lp->m, dk, lp->cq, pdq, done, st) !=
        lp->cg_nf)
      return set_error("fused CG: finish shape mismatch"), SKIPM_EINVAL;
  }
  ColPass pq = cg_close_args(lp, xsol, iter & 1);
  pq.cg.k = iter;
  SK_TRY(run_colpass(pq, st));
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

// Small dense LPs: the whole CG in one workgroup (one launch, one host read).
// Returns 1 if it ran, 0 if this LP takes the multi-workgroup path.
int pcg_small(skipm_lp_s* lp, const double* rhs, double* xsol, double tol, int max_it,
              int* its, int* fact_fail, hipStream_t st) {
  if (lp->fmt != SKIPM_DENSE || lp->small_cg_bytes <= 0 || lp->tier == SKIPM_TIER_BF16) return 0;
  const bool f32 = lp->tier == SKIPM_TIER_FP32;
  const int ta = f32 ? SKIPM_F32 : lp->a_dtype;
  const int64_t bytes = lp->lda * lp->n * (ta == SKIPM_F64 ? 8 : 4);
  if (bytes > lp->small_cg_bytes) return 0;
  SmallCg a;
  a.A = f32 ? (const void*)lp->A32 : lp->A;
  a.lda = lp->lda;
  a.m = lp->m;
  a.n = lp->n;
  a.d2 = lp->d2;
  a.Qi = lp->G;
  a.mp = lp->mp;
  a.rhs = rhs;
  a.x = xsol;
  a.r = lp->cr;
  a.z = lp->cz;
  a.d = lp->cd;
  a.sc = lp->sc;
  a.is = lp->is;
  a.tol = tol;
  a.max_it = max_it;
  a.inner = lp->prm.inner;
  if (launch_cg_small(a, ta, st) != 0) return 0;
  if (hipGetLastError() != hipSuccess) return set_error("small CG launch failed"), SKIPM_EDEVICE;
  if (sync_read(lp, st) != SKIPM_OK) return SKIPM_EDEVICE;
  const int32_t* hi = host_ints(lp);
  *fact_fail = hi[I_FACT_FAIL] ? 1 : 0;
  *its = hi[I_CG_ITERS];
  return 1;
}

// CG iterations are enqueued in chunks, each followed by an asynchronous copy
// of the scalar block into one of two pinned snapshots.  While the host waits
// for one snapshot, the next chunk is already queued, so the device does not
// wait for the host's check; what it costs is the chunk queued behind the one
// in which CG stops (its passes read the done flag and return).  So chunks
// shrink towards the stop: the stopping quantity (r^T z, or r^T r) falls by a
// factor c_prev / c_k over the last k - k_prev iterations, and at that rate
// reaches c_stop after about (k - k_prev) log(c_k / c_stop) / log(c_prev / c_k)
// more; the next chunk is half of what that leaves beyond the queued
// iterations, between 1 and kCgChunkMax.  (CG converges faster towards the
// end, so the recent rate, halved, rarely overshoots.)  LPs solved next to
// others (the batch and the request server) keep one snapshot in flight: the
// host checks each chunk with the stream idle, as the others' work fills the
// device meanwhile.
constexpr int kCgChunkDefault = 4, kCgChunkMax = 16;

struct CgProgress {
  int k = 0;       // CG iteration of the last snapshot read
  double c = -1;   // its stopping quantity (negative: none yet)
};

int next_cg_chunk(const double* snap, int enq, CgProgress* last) {
  const int32_t* hi = (const int32_t*)(snap + S_NSLOTS);
  const int k = hi[I_CG_ITERS];
  const bool resid = hi[I_CG_RESID] != 0;
  const double ck = resid ? snap[S_V_RR] : snap[S_CG_RZ];
  const double cs = snap[S_CG_TOL2];
  const CgProgress prev = last->c < 0 ? CgProgress{0, resid ? snap[S_V_GG] : snap[S_CG_RZ0]}
                                      : *last;
  last->k = k;
  last->c = ck;
  if (!(k > prev.k && cs > 0 && ck > cs && prev.c > ck)) return kCgChunkDefault;
  const double need = (k - prev.k) * log(ck / cs) / log(prev.c / ck);
  const double half = 0.5 * (need - (enq - k));  // half of what lies beyond the queue
  if (!(half < kCgChunkMax)) return kCgChunkMax;
  return std::max(1, (int)half);
}

// CG on A D^2 A^T dy = rhs preconditioned by Q^{-1}; returns iterations in *its.
// The snapshot the host stops on is the final state: passes after the stop
// change nothing.
int pcg_run(skipm_lp_s* lp, const double* rhs, double* xsol, double tol, int max_it,
            int first_chunk, int* its, int* fact_fail, hipStream_t st) {
  {
    const int rc = pcg_small(lp, rhs, xsol, tol, max_it, its, fact_fail, st);
    if (rc < 0) return rc;
    if (rc == 1) return SKIPM_OK;
  }
  SK_TRY(qinv_apply(lp, rhs, lp->cw, nullptr, st));
  launch_cg_init(lp->m, rhs, lp->cw, lp->cr, lp->cz, lp->cd, nullptr, xsol, nullptr, 0, lp->sc,
                 lp->is, tol, max_it, 0, st);
  *fact_fail = 0;
  int enq = 0, slot = 0;
  int queue[2], nq = 0;  // snapshots in flight, oldest first
  bool capped[2] = {false, false};
  // snapshots in flight: two overlap the check with the next chunk; one checks
  // each chunk with the stream idle (a plain stream synchronisation)
  const int depth = lp->overlap_checks ? 2 : 1;
  auto enqueue = [&](int n) -> int {
    for (int q = 0; q < n && enq < max_it; ++q, ++enq) SK_TRY(pcg_iteration(lp, xsol, enq, st));
    capped[slot] = enq >= max_it;
    if (capped[slot])  // close the capped run (the next iteration's opening pass would)
      launch_cg_close(lp->cgred + lp->cg_nf, lp->cg_nd, enq, lp->sc, lp->is, st);
    SK_CHECK_HIP(hipMemcpyAsync(lp->hsnap[slot], lp->sc, kScalarBlockBytes,
                                hipMemcpyDeviceToHost, st));
    if (depth == 2) SK_CHECK_HIP(hipEventRecord(lp->snap_ev[slot], st));
    queue[nq++] = slot;
    slot ^= 1;
    return SKIPM_OK;
  };
  SK_TRY(enqueue(std::max(1, std::min(first_chunk, max_it))));
  int next = std::min(kCgChunkDefault, std::max(1, first_chunk));
  CgProgress progress;
  for (;;) {
    if (nq < depth && enq < max_it) {
      SK_TRY(enqueue(next));
    }
    const int look = queue[0];
    queue[0] = queue[1];
    --nq;
    if (depth == 2) {
      SK_TRY(poll_event(lp->snap_ev[look]));
    } else {
      SK_TRY(wait_stream(st, lp->rd_ev));
    }
    const double* snap = lp->hsnap[look];
    const int32_t* hi = (const int32_t*)(snap + S_NSLOTS);
    const bool fail = hi[I_FACT_FAIL] != 0;
    const bool stop = fail || hi[I_CG_DONE] || capped[look];
    kt_harvest(lp, fail ? 0 : hi[I_CG_ITERS], stop);
    if (stop) {
      memcpy(lp->hsc, snap, kScalarBlockBytes);
      *fact_fail = fail ? 1 : 0;
      *its = hi[I_CG_ITERS];
      return SKIPM_OK;
    }
    next = next_cg_chunk(snap, enq, &progress);
  }
}

// First chunk of a CG run: two thirds of the previous normal-equation solve's
// iteration count, since a short first chunk costs only overlapped checks
// while a long one enqueues passes past the stop (the counts of successive IPM
// iterations often fall by a quarter or more).  Refinement steps after the
// first correct only the rounding of A's copy and take few iterations: they
// start with two.
int first_cg_chunk(const skipm_lp_s* lp, int outer) {
  return outer == 0 ? std::max(2, lp->prev_cg * 2 / 3) : 2;
}

// FP64 residual of the normal equations, rt = rhs - A D^2 A^T x (one FP64 pass
// over A), and S_RHO2 = rt^T Q^{-1} rt.
int normal_residual_fp64(skipm_lp_s* lp, const double* rhs, const double* x, hipStream_t st) {
  if (lp->fmt == SKIPM_CSR) {
    SK_TRY(normal_sparse(lp, x, -1.0, rhs, 1.0, lp->rt, nullptr, st));
  } else {
    ColPass cp = colpass_A(lp, COL_NORMAL);
    cp.u = x;
    cp.d2 = lp->d2;
    SK_TRY(run_colpass(cp, st));
    launch_finish(lp->part, lp->mp, 0, cp.nblk, lp->m, -1.0, rhs, 1.0, lp->rt,
                  nullptr, st);
  }
  SK_TRY(qinv_apply(lp, lp->rt, lp->uv1, nullptr, st));
  launch_dot(lp->rt, lp->uv1, lp->m, lp->sc, S_RHO2, st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

// Outer refinement steps after which the current tier's copy of A counts as
// too coarse for this iterate (kappa(A D) too large): the rest of this solve,
// and of the run, takes the products one tier up.
constexpr int kRefineMaxOuter = 4;
constexpr int kRefineCap = 8;

// One precision tier up (BF16 -> FP32 -> FP64); records the first move.
void escalate_tier(skipm_lp_s* lp) {
  if (lp->tier == SKIPM_TIER_FP64) return;
  lp->tier = lp->tier == SKIPM_TIER_BF16 ? SKIPM_TIER_FP32 : SKIPM_TIER_FP64;
  if (lp->demote_iter < 0) lp->demote_iter = (int)lp->k;
}

// Mixed precision: iterative refinement with FP64 residuals around a CG whose
// products read the current tier's low-precision copy of A (FP64
// accumulation).  Stops on the same test as the FP64 CG,
// sqrt(r^T Q^{-1} r) <= tol sqrt(p^T Q^{-1} p), with r the FP64 residual, or
// once the inner runs together have taken max_it CG iterations.
int pcg_refined(skipm_lp_s* lp, const double* rhs, double* xsol, double tol, int max_it,
                int* its, int* fact_fail, hipStream_t st) {
  launch_fill_f64(xsol, 0.0, lp->m, st);
  launch_copy_f64(lp->rt, rhs, lp->m, st);
  double rho0 = -1, rho = 0;
  int total = 0;
  *fact_fail = 0;
  int outer = 0;
  for (; outer < kRefineCap; ++outer) {
    const int budget = max_it - total;
    if (budget <= 0) break;  // the solve's CG cap is spent
    // The inner CG is consistent (FP64 accumulation), so it can go straight to
    // the target; further outer steps only correct the rounding of A's copy.
    const double rel_target = rho0 > 0 && rho > 0 ? tol * rho0 / rho : tol;
    const double inner_tol = std::min(0.5, rel_target);
    int inner = 0;
    const int first = first_cg_chunk(lp, outer);
    SK_TRY(pcg_run(lp, lp->rt, lp->dyc, tol > 0 ? inner_tol : 0.0, budget, first, &inner,
                   fact_fail, st));
    if (*fact_fail) return SKIPM_OK;
    if (outer + 1 >= kRefineMaxOuter) escalate_tier(lp);
    if (rho0 < 0) rho0 = sqrt(std::max(0.0, lp->hsc[S_CG_RZ0]));
    total += inner;
    launch_axpy(xsol, lp->dyc, 1.0, lp->m, st);
    SK_TRY(normal_residual_fp64(lp, rhs, xsol, st));
    SK_TRY(sync_read(lp, st));
    rho = sqrt(std::max(0.0, lp->hsc[S_RHO2]));
    if (!(rho0 > 0) || rho <= tol * rho0 || tol <= 0) {
      ++outer;
      break;
    }
  }
  lp->last_outer = std::max(outer, 1);
  // report the FP64 residual in the CG slots
  lp->hsc[S_CG_RZ0] = rho0 * rho0;
  lp->hsc[S_CG_RZ] = rho * rho;
  *its = total;
  return SKIPM_OK;
}

int sketch_into(skipm_lp_s* lp, const double* dscale, int is_d2, int64_t salt, double* B,
                hipStream_t st);

// Alg. 1 for one right-hand side: the sketch B = A D W with this salt, Q^{-1}
// from its Gram matrix, then CG.  A non-positive pivot of the Gram matrix is
// Lemma 3's failure event (rank(A D W) < m): the sketch is drawn again with a
// fresh salt, up to kFreshSketches times.  If every sketch fails, A D itself
// is numerically rank deficient and the last sketch's Gram matrix is factored
// with a growing relative diagonal shift (kShifts times) before SKIPM_ERANK.
constexpr int kFreshSketches = 3, kShifts = 3;

int sketch_solve(skipm_lp_s* lp, const double* dscale, int is_d2, int64_t salt,
                 const double* rhs, double* xsol, double tol, int max_it, int* its,
                 hipStream_t st, int first_attempt = 0) {
  if (first_attempt == 0) {
    lp->step_resketches = 0;
    lp->step_shifts = 0;
  }
  lp->last_outer = 1;
  double shift = 0.0;
  int rc = SKIPM_ERANK;
  for (int attempt = first_attempt; attempt <= kFreshSketches + kShifts; ++attempt) {
    if (attempt <= kFreshSketches) {
      // fresh salts sit far above any IPM iteration index
      const int64_t sa = salt + ((int64_t)attempt << 40);
      SK_TRY(sketch_into(lp, dscale, is_d2, sa, lp->B, st));
      if (attempt > 0) ++lp->step_resketches;
    } else {
      shift = shift == 0.0 ? 1e-12 : shift * 1e3;
      ++lp->step_shifts;
    }
    SK_TRY(factor(lp, shift, st));
    int fail = 0;
    if (lp->tier != SKIPM_TIER_FP64) {
      SK_TRY(pcg_refined(lp, rhs, xsol, tol, max_it, its, &fail, st));
    } else {
      SK_TRY(pcg_run(lp, rhs, xsol, tol, max_it, first_cg_chunk(lp, 0), its, &fail, st));
    }
    if (!fail) {
      rc = SKIPM_OK;
      break;
    }
  }
  lp->run_resketches += lp->step_resketches;
  lp->run_shifts += lp->step_shifts;
  if (rc != SKIPM_OK)
    set_error("the sketch's Gram matrix kept a non-positive pivot through fresh sketches and "
              "diagonal shifts (rank(A D W) < m)");
  return rc;
}

int gaussian_ready(skipm_lp_s* lp) {
  lp->ldw = round_up(lp->n, 2);
  if (!lp->Wd) SK_TRY(dalloc(lp, &lp->Wd, lp->ldw * (int64_t)lp->w));
  if (!lp->gy) SK_TRY(dalloc(lp, &lp->gy, lp->n));
  return SKIPM_OK;
}

int sketch_into(skipm_lp_s* lp, const double* dscale, int is_d2, int64_t salt, double* B,
                hipStream_t st) {
  if (lp->prm.sketch == SKIPM_SKETCH_GAUSSIAN) {
    // B = A (D W_G): fill D W_G, then the FP64 matrix-core GEMM over the padded
    // rows, split along n into slices that are summed in order
    SK_TRY(gaussian_ready(lp));
    launch_gauss_fill(lp->prm.seed, salt, lp->n, lp->w, dscale, is_d2, lp->Wd, lp->ldw, st);
    SK_CHECK_HIP(hipGetLastError());
    const double* A = (const double*)lp->A;
    const int ns = gauss_gemm_slices(lp->n, gauss_ksplit(lp->lda, lp->w, lp->n));
    const bool timed = lp->kt_every > 0 && lp->ks_ev[0] && !lp->ks_pending &&
                       hipEventRecord(lp->ks_ev[0], st) == hipSuccess;
    if (ns <= 1) {
      launch_gauss_gemm(A, lp->lda, lp->Wd, lp->ldw, lp->w, lp->n, 1, B, st);
    } else {
      const int64_t lw = lp->lda * (int64_t)lp->w;
      if (!lp->Bsplit) SK_TRY(dalloc(lp, &lp->Bsplit, (int64_t)gauss_ksplit(lp->lda, lp->w, lp->n) * lw));
      launch_gauss_gemm(A, lp->lda, lp->Wd, lp->ldw, lp->w, lp->n, ns, lp->Bsplit, st);
      launch_sum_slices(lp->Bsplit, ns, lw, B, st);
    }
    SK_CHECK_HIP(hipGetLastError());
    if (timed) lp->ks_pending = hipEventRecord(lp->ks_ev[1], st) == hipSuccess;
    return SKIPM_OK;
  }
  SK_TRY(hash_items(lp, salt, st));
  const bool timed = lp->kt_every > 0 && lp->ks_ev[0] && !lp->ks_pending &&
                     hipEventRecord(lp->ks_ev[0], st) == hipSuccess;
  if (lp->fmt == SKIPM_CSR)
    launch_sketch_csc(lp->sp, lp->s, dscale, is_d2, lp->bptr, lp->perm, lp->sign, lp->w, B,
                      lp->lda, st);
  else
    launch_sketch_dense(lp->A, lp->a_dtype, lp->lda, lp->m, lp->n, lp->s, dscale, is_d2,
                        lp->bptr, lp->perm, lp->sign, lp->w, B, lp->lda, st);
  SK_CHECK_HIP(hipGetLastError());
  if (timed) lp->ks_pending = hipEventRecord(lp->ks_ev[1], st) == hipSuccess;
  return SKIPM_OK;
}

// adds the pending sketch-product sample once its end event has completed
void ks_harvest(skipm_lp_s* lp) {
  if (!lp->ks_pending) return;
  float ms = 0;
  if (hipEventQuery(lp->ks_ev[1]) == hipSuccess &&
      hipEventElapsedTime(&ms, lp->ks_ev[0], lp->ks_ev[1]) == hipSuccess) {
    lp->ks_sum_ms += ms;
    ++lp->ks_count;
    lp->ks_pending = false;
  }
}

int epilogue(skipm_lp_s* lp, hipStream_t st) {
  if (lp->fmt == SKIPM_CSR) {
    const SparseA& A = lp->sp;
    if (launch_csc_dot(A, COL_EPILOGUE, lp->dy, nullptr, nullptr, nullptr, lp->rd, lp->d2,
                       lp->cf1, nullptr, nullptr, nullptr, lp->ds, nullptr, lp->sc, nullptr,
                       lp->nblk_csc, st) != 0)
      return set_error("m too large for the sparse path"), SKIPM_EINVAL;
    launch_csr_segsum(A, lp->cf1, nullptr, lp->segsum, nullptr, st);
    launch_csr_fold(A, lp->segsum, 0, 1.0, lp->p, -1.0, lp->g, nullptr, st);
    SK_CHECK_HIP(hipGetLastError());
    return SKIPM_OK;
  }
  ColPass cp = colpass_A(lp, COL_EPILOGUE);
  cp.u = lp->dy;
  cp.rd = lp->rd;
  cp.d2 = lp->d2;
  cp.ds_out = lp->ds;
  SK_TRY(run_colpass(cp, st));
  // g = A D^2 A^T dy - p
  launch_finish(lp->part, lp->mp, 0, cp.nblk, lp->m, 1.0, lp->p, -1.0, lp->g, nullptr,
                st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

// ---- correction vector: t = (A D W)^+ g ---------------------------------------
//
// eq. compv needs t = B^+ g with B = A D W, so that B t = g holds to working
// accuracy (it is what keeps the residuals on their segment, eq. addl).  Late in
// the IPM kappa(B) reaches 1e8 and anything that goes through the FP64 Gram
// matrix B B^T alone loses the residual.  So t is refined on the true residual
// r = g - B t (formed from B itself), with an inner approximate pseudo-inverse
// taken from Cholesky-QR rounds on B: round 0 uses P0 = (B B^T)^{-1} (the CG
// preconditioner), round K >= 1 the whitened B_K = L_{K-1}^{-1} ... L_0^{-1} B,
// whose Gram matrix is well conditioned.  Rounds are built only when the
// refinement contracts poorly.

int alloc_vbuffers(skipm_lp_s* lp) {
  if (lp->B1) return SKIPM_OK;
  const int64_t lw = lp->lda * lp->w, mm = lp->mp * lp->mp;
  SK_TRY(dalloc(lp, &lp->B1, lw));
  SK_TRY(dalloc(lp, &lp->B2, lw));
  SK_TRY(dalloc(lp, &lp->Gv, mm));
  SK_TRY(dalloc(lp, &lp->Xv, mm));
  SK_TRY(dalloc(lp, &lp->M1, mm));
  SK_TRY(dalloc(lp, &lp->M2, mm));
  return SKIPM_OK;
}

// out(m) = Mat(mp x mp, column-major) * u, Mat lower triangular (AXPY pass + finish)
int tri_apply(skipm_lp_s* lp, const double* Mat, const double* u, double* out, hipStream_t st) {
  ColPass cp{};
  cp.mode = COL_AXPY;
  cp.A = Mat;
  cp.ta = SKIPM_F64;
  cp.tc = SKIPM_F64;
  cp.lda = lp->mp;
  cp.m = lp->m;
  cp.n = lp->m;
  cp.d2 = u;
  cp.part = lp->part;
  cp.ldp = lp->mp;
  cp.nblk = 0;
  SK_TRY(run_colpass(cp, st));
  launch_finish(lp->part, lp->mp, 0, cp.nblk, lp->m, 1.0, nullptr, 0.0, out, nullptr,
                st);
  return SKIPM_OK;
}

// out(mp) = Sym(mp x mp) u  (DOT pass over the symmetric matrix's columns)
int sym_apply(skipm_lp_s* lp, const double* Sym, const double* u, double* out, hipStream_t st) {
  ColPass cp{};
  cp.mode = COL_DOT;
  cp.A = Sym;
  cp.ta = SKIPM_F64;
  cp.tc = SKIPM_F64;
  cp.lda = lp->mp;
  cp.m = lp->mp;
  cp.n = lp->m;
  cp.u = u;
  cp.t_out = out;
  cp.nblk = 0;
  return run_colpass(cp, st);
}

// out(w) = Bk^T u
int sketch_t_apply(skipm_lp_s* lp, const double* Bk, const double* u, double* out,
                   hipStream_t st) {
  ColPass cp{};
  cp.mode = COL_DOT;
  cp.A = Bk;
  cp.ta = SKIPM_F64;
  cp.tc = SKIPM_F64;
  cp.lda = lp->lda;
  cp.m = lp->m;
  cp.n = lp->w;
  cp.u = u;
  cp.t_out = out;
  cp.nblk = 0;
  return run_colpass(cp, st);
}

// out = g - B t ; S_V_RR = ||out||^2
int true_residual(skipm_lp_s* lp, const double* t, double* out, hipStream_t st) {
  ColPass cp{};
  cp.mode = COL_AXPY;
  cp.A = lp->B;
  cp.ta = SKIPM_F64;
  cp.tc = SKIPM_F64;
  cp.lda = lp->lda;
  cp.m = lp->m;
  cp.n = lp->w;
  cp.d2 = t;
  cp.part = lp->part;
  cp.ldp = lp->mp;
  cp.nblk = lp->nblk_B;
  SK_TRY(run_colpass(cp, st));
  launch_finish(lp->part, lp->mp, 0, cp.nblk, lp->m, -1.0, lp->g, 1.0, out, nullptr, st);
  launch_norm2(out, lp->m, lp->sc, S_V_RR, st);
  return SKIPM_OK;
}

int spd_inverse_checked(skipm_lp_s* lp, double* Gm, double* Xm, hipStream_t st) {
  launch_fill_f64_flag(Xm, 0.0, lp->mp * lp->mp, lp->is + I_FACT_FAIL, st);
  launch_spd_inverse(Gm, Xm, lp->Ct, lp->mp, lp->is + I_FACT_FAIL, st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

// Build round K (1 or 2) of the whitening.  *ok = 0 when neither the round's
// Gram matrix nor its shifted form has a Cholesky factor (the round is unusable).
int build_vround(skipm_lp_s* lp, int K, int* ok, hipStream_t st) {
  SK_TRY(alloc_vbuffers(lp));
  const int64_t mp = lp->mp, mm = mp * mp;
  if (K == 1) {
    launch_copy_f64(lp->M1, lp->Xb, mm, st);  // M1 = X0
    launch_trmm(lp->Xb, mp, lp->B, lp->lda, lp->m, lp->w, lp->B1, lp->lda, lp->lda, st);
    launch_gram(lp->B1, lp->lda, lp->m, lp->w, lp->Gpart, lp->ksplit, mp, st);
  } else {
    launch_trmm(lp->Xv, mp, lp->B1, lp->lda, lp->m, lp->w, lp->B2, lp->lda, lp->lda, st);
    launch_trmm(lp->Xv, mp, lp->M1, mp, mp, mp, lp->M2, mp, mp, st);  // M2 = X1 M1
    launch_gram(lp->B2, lp->lda, lp->m, lp->w, lp->Gpart, lp->ksplit, mp, st);
  }
  launch_gram_finish(lp->Gpart, lp->ksplit, lp->m, mp, lp->Gv, st);
  SK_TRY(spd_inverse_checked(lp, lp->Gv, lp->Xv, st));
  SK_TRY(sync_read(lp, st));
  if (host_ints(lp)[I_FACT_FAIL]) {
    // shifted Cholesky of the round's Gram matrix
    launch_gram_finish(lp->Gpart, lp->ksplit, lp->m, mp, lp->Gv, st);
    launch_shift_trace(lp->Gv, mp, lp->m, 11.0 * (double)(lp->w * lp->m + lp->m * (lp->m + 1)) *
                                              1.1102230246251565e-16, st);
    SK_TRY(spd_inverse_checked(lp, lp->Gv, lp->Xv, st));
    SK_TRY(sync_read(lp, st));
    if (host_ints(lp)[I_FACT_FAIL]) {
      *ok = 0;
      return SKIPM_OK;
    }
  }
  lp->vrounds_built = K;
  *ok = 1;
  return SKIPM_OK;
}

// tq = approximate B^+ rv from round K
int pinv_apply(skipm_lp_s* lp, int K, hipStream_t st) {
  if (K == 0) {
    SK_TRY(sym_apply(lp, lp->G, lp->rv, lp->uv2, st));
    return sketch_t_apply(lp, lp->B, lp->uv2, lp->tq, st);
  }
  SK_TRY(tri_apply(lp, K == 1 ? lp->M1 : lp->M2, lp->rv, lp->uv1, st));
  SK_TRY(sym_apply(lp, lp->Gv, lp->uv1, lp->uv2, st));
  return sketch_t_apply(lp, K == 1 ? lp->B1 : lp->B2, lp->uv2, lp->tq, st);
}

// t = (A D W)^+ g by refinement (policy in vrefine.h).  Each step forms the
// candidate t' = t + P (g - B t) and its true residual beside the kept t, and
// keeps it only if its residual is finite and smaller, so the t that eq. compv
// turns into v is always the best one found.  A non-finite g (nothing to
// refine against) is reported as SKIPM_ENAN.
int v_solve(skipm_lp_s* lp, int* its, double* rel_out, hipStream_t st) {
  lp->vrounds_built = 0;
  launch_v_init(lp->tw, lp->w, lp->rv, lp->g, lp->m, lp->sc, S_V_GG, st);  // t = 0, r = g
  *its = 0;
  *rel_out = 0.0;
  VRefine pol;
  // ||g||^2 is read with the first step's residual (one host read fewer); a
  // zero g gives t = 0 without refinement, as if tested first
  for (;;) {
    SK_TRY(pinv_apply(lp, pol.round, st));
    launch_add_f64(lp->tw2, lp->tw, lp->tq, lp->w, st);
    SK_TRY(true_residual(lp, lp->tw2, lp->rv2, st));
    SK_CHECK_HIP(hipGetLastError());
    SK_TRY(sync_read(lp, st));
    const double gg = lp->hsc[S_V_GG];
    if (!std::isfinite(gg)) {
      set_error("non-finite residual g of the normal equations");
      return SKIPM_ENAN;
    }
    if (!(gg > 0.0)) return SKIPM_OK;  // g = 0: t stays 0
    const double rr = lp->hsc[S_V_RR];
    const double rel = std::isfinite(rr) && rr >= 0.0 ? sqrt(rr / gg) : NAN;
    bool keep = false;
    const VAct act = v_refine_next(pol, rel, &keep);
    if (keep) {
      std::swap(lp->tw, lp->tw2);
      std::swap(lp->rv, lp->rv2);
    }
    *its = pol.steps;
    *rel_out = pol.best;
    if (act == V_STOP) break;
    if (act == V_BUILD) {
      int ok = 0;
      SK_TRY(build_vround(lp, pol.round, &ok, st));
      if (!ok) break;  // no better pseudo-inverse: keep the best t
    }
  }
  return SKIPM_OK;
}

int finish_step(skipm_lp_s* lp, hipStream_t st) {
  const double* wt = nullptr;
  if (lp->prm.sketch == SKIPM_SKETCH_GAUSSIAN) {
    // (D W_G) t; the direction kernel forms v_j = sqrt(x_j s_j) (W_G t)_j = s_j (D W_G t)_j
    launch_gauss_gemv(lp->Wd, lp->ldw, lp->n, lp->w, lp->tw, lp->gy, st);
    SK_CHECK_HIP(hipGetLastError());
    wt = lp->gy;
  }
  if (lp->nblk_vec == 1 && lp->step_one) {
    launch_step_one(lp->n, lp->m, lp->s, lp->x, lp->y, lp->sv, lp->d2, lp->ds, lp->dy, lp->bucket,
                    lp->sign, lp->tw, wt, lp->v, lp->dx, lp->sc, st);
    SK_CHECK_HIP(hipGetLastError());
    return SKIPM_OK;
  }
  launch_direction(lp->n, lp->s, lp->x, lp->sv, lp->d2, lp->ds, lp->bucket, lp->sign, lp->tw,
                   wt, lp->v, lp->dx, lp->red, lp->nblk_vec, lp->sc, st);
  launch_reduce_slots(lp->red, lp->nblk_vec, 5, lp->sc, S_A0, 0, st);
  launch_step_terms(lp->n, lp->x, lp->sv, lp->dx, lp->ds, lp->red, lp->nblk_vec, lp->sc, st);
  launch_reduce_slots(lp->red, lp->nblk_vec, 2, lp->sc, S_EXIT, 1, st);
  launch_step_finalize(lp->n, lp->sc, st);
  launch_update(lp->n, lp->m, lp->x, lp->y, lp->sv, lp->dx, lp->dy, lp->ds, lp->red, lp->nblk_vec,
                lp->sc, st);
  launch_mu_finalize(lp->red, lp->nblk_vec, lp->n, lp->sc, st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}

struct StopState {
  bool converged;
  bool nan;
  double ctx, bty, rel_gap, rp, rd, mu;
};

StopState stop_test(skipm_lp_s* lp, double bnorm, double cnorm) {
  const double* h = lp->hsc;
  StopState s{};
  s.ctx = h[S_CTX];
  s.bty = h[S_BTY];
  s.mu = h[S_MU];
  s.rp = sqrt(h[S_RP2]);
  s.rd = sqrt(h[S_RD2]);
  const double den = std::max(1.0, fabs(s.ctx));
  s.rel_gap = fabs(s.ctx - s.bty) / den;
  s.nan = !(std::isfinite(s.ctx) && std::isfinite(s.bty) && std::isfinite(s.mu) &&
            std::isfinite(s.rp) && std::isfinite(s.rd));
  s.converged = !s.nan && s.rel_gap <= lp->prm.eps_gap && h[S_XS] <= lp->prm.eps_gap * den &&
                s.rp <= lp->prm.eps_feas * bnorm && s.rd <= lp->prm.eps_feas * cnorm;
  return s;
}

int step_internal(skipm_lp_s* lp, skipm_step_info* info, double bnorm, double cnorm,
                  hipStream_t st) {
  SK_TRY(prologue(lp, st));
  // Far from convergence the stopping test's slots are read at the CG's first
  // host check: the sketch, the factorisation and the CG are queued behind
  // the prologue without a host round trip of their own (none of them writes
  // those slots), and a failure there counts only if the iterate has not
  // converged.  Once the last relative gap is within 16 eps_gap (mu shrinks
  // by at most 1 - alpha (1 - sigma) >= 1/2 per step, so the test can pass
  // only then) the test is read first, so the final iteration queues nothing.
  const bool defer = lp->last_rel_gap > 16.0 * lp->prm.eps_gap;
  const int64_t salt = lp->prm.resketch ? lp->k : 0;
  int its = 0;
  int rc = SKIPM_OK;
  if (defer) {
    rc = sketch_solve(lp, lp->d2, 1, salt, lp->p, lp->dy, lp->prm.tol_cg, lp->prm.max_cg, &its,
                      st);
  }
  if (!defer || rc != SKIPM_OK) SK_TRY(sync_read(lp, st));
  // the prologue's x^T s is the same quantity as the update's; S_XS holds the
  // value of the current iterate
  const StopState ss = stop_test(lp, bnorm, cnorm);
  lp->last_rel_gap = ss.nan ? HUGE_VAL : ss.rel_gap;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->mu = ss.mu;
    info->rp_norm = ss.rp;
    info->rd_norm = ss.rd;
    info->rel_gap = ss.rel_gap;
    info->eta = lp->hsc[S_ETA];
    info->tier = lp->tier;
  }
  if (ss.nan) {
    set_error("non-finite iterate");
    if (info) info->status = SKIPM_ENAN;
    return SKIPM_ENAN;
  }
  if (lp->k > 0) {  // step length of the previous iteration
    lp->small_steps = lp->hsc[S_ALPHA] < 1e-12 ? lp->small_steps + 1 : 0;
    if (lp->small_steps >= 3) {
      set_error("step length below 1e-12 three times in a row");
      if (info) info->status = SKIPM_ESTALL;
      return SKIPM_ESTALL;
    }
  }
  if (ss.converged) {
    if (info) info->converged = 1;
    return SKIPM_OK;
  }
  if (!defer)
    rc = sketch_solve(lp, lp->d2, 1, salt, lp->p, lp->dy, lp->prm.tol_cg, lp->prm.max_cg, &its,
                      st);
  if (info) {
    info->tier = lp->tier;
    info->refine_steps = lp->last_outer;
    info->resketches = lp->step_resketches;
    info->shifts = lp->step_shifts;
  }
  if (rc != SKIPM_OK) {
    if (info) info->status = rc;
    return rc;
  }
  ks_harvest(lp);  // the CG's host checks have waited past the sketch
  const double f0 = sqrt(std::max(0.0, lp->hsc[S_CG_RZ0]));
  const double f1 = sqrt(std::max(0.0, lp->hsc[S_CG_RZ]));
  lp->prev_cg = its;
  SK_TRY(epilogue(lp, st));
  int vits = 0;
  double vrel = 0;
  rc = v_solve(lp, &vits, &vrel, st);
  if (rc != SKIPM_OK) {
    if (info) info->status = rc;
    return rc;
  }
  SK_TRY(finish_step(lp, st));
  lp->k += 1;
  if (info) {
    info->cg_iters = its;
    info->f0_norm = f0;
    info->f_norm = f1;
    info->v_iters = vits;
    info->v_resid = vrel;
  }
  return SKIPM_OK;
}

// res from the slots of the last stopping test (the rest of res, the CG
// counts, is accumulated by the caller)
void fill_result(skipm_lp_s* lp, skipm_result* res, int status, int it) {
  const StopState ss = stop_test(lp, lp->bnorm, lp->cnorm);
  res->status = status;
  res->iters = it;
  res->obj_p = ss.ctx;
  res->obj_d = ss.bty;
  res->rel_gap = ss.rel_gap;
  res->rp_norm = ss.rp;
  res->rd_norm = ss.rd;
  res->mu = ss.mu;
  res->demote_iter = lp->demote_iter;
  res->tier_final = lp->tier;
  res->resketches = lp->run_resketches;
  res->shifts = lp->run_shifts;
}

double host_norm(const double* dptr, int64_t n, int* rc) {
  std::vector<double> h((size_t)n);
  if (hipMemcpy(h.data(), dptr, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    *rc = SKIPM_EDEVICE;
    return 0;
  }
  double s = 0;
  for (double v : h) s += v * v;
  *rc = SKIPM_OK;
  return sqrt(s);
}

}  // namespace

namespace skipm {

bool batch_groupable(const skipm_lp_s* lp) {
  return lp->fmt == SKIPM_DENSE && lp->start_tier == SKIPM_TIER_FP64;
}

void batch_phase_a(skipm_lp_s* lp, skipm_result* res, BatchLp* b, hipStream_t st) {
  b->grouped = false;
  b->its = 0;
  b->fail = 0;
  auto end = [&](int status) {
    fill_result(lp, res, status, b->it);
    b->active = false;
  };
  auto check = [&](int rc) {
    if (rc == SKIPM_OK) return true;
    b->rc = rc;
    b->err = skipm_last_error();
    res->status = rc;
    b->active = false;
    return false;
  };
  if (!check(hipSetDevice(lp->device) == hipSuccess ? SKIPM_OK : SKIPM_EDEVICE)) return;
  if (!check(prologue(lp, st)) || !check(sync_read(lp, st))) return;
  const StopState ss = stop_test(lp, lp->bnorm, lp->cnorm);
  lp->last_rel_gap = ss.nan ? HUGE_VAL : ss.rel_gap;
  if (b->it >= lp->prm.max_outer) {
    end(ss.converged ? SKIPM_OK : (ss.nan ? SKIPM_ENAN : SKIPM_ENOTCONV));
    return;
  }
  if (ss.nan) return end(SKIPM_ENAN);
  if (lp->k > 0) {
    lp->small_steps = lp->hsc[S_ALPHA] < 1e-12 ? lp->small_steps + 1 : 0;
    if (lp->small_steps >= 3) return end(SKIPM_ESTALL);
  }
  if (ss.converged) return end(SKIPM_OK);
  const int64_t salt = lp->prm.resketch ? lp->k : 0;
  lp->step_resketches = 0;
  lp->step_shifts = 0;
  lp->last_outer = 1;
  if (!check(sketch_into(lp, lp->d2, 1, salt, lp->B, st)) || !check(factor(lp, 0.0, st))) return;
  // the one-workgroup CG where pcg_run would take it (small dense FP64 LPs),
  // else the grouped CG
  const int rc = pcg_small(lp, lp->p, lp->dy, lp->prm.tol_cg, lp->prm.max_cg, &b->its, &b->fail, st);
  if (rc < 0) check(rc);
  else b->grouped = rc == 0;
}

void batch_phase_b(skipm_lp_s* lp, skipm_result* res, BatchLp* b, hipStream_t st) {
  auto fail_with = [&](int rc) {
    if (rc == SKIPM_EINVAL || rc == SKIPM_EDEVICE || rc == SKIPM_ENOMEM) {
      b->rc = rc;
      b->err = skipm_last_error();
    }
    fill_result(lp, res, rc, b->it);
    b->active = false;
  };
  if (hipSetDevice(lp->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return fail_with(SKIPM_EDEVICE);
  }
  int its = b->its;
  if (b->fail) {
    // Lemma 3's failure event: fresh sketches, then shifts, each with its own CG
    const int64_t salt = lp->prm.resketch ? lp->k : 0;
    const int rc = sketch_solve(lp, lp->d2, 1, salt, lp->p, lp->dy, lp->prm.tol_cg,
                                lp->prm.max_cg, &its, st, 1);
    if (rc != SKIPM_OK) return fail_with(rc);
  } else {
    lp->run_resketches += lp->step_resketches;
    lp->run_shifts += lp->step_shifts;
  }
  lp->prev_cg = its;
  res->cg_total += its;
  res->cg_max = std::max(res->cg_max, its);
  int rc = epilogue(lp, st);
  if (rc != SKIPM_OK) return fail_with(rc);
  int vits = 0;
  double vrel = 0;
  rc = v_solve(lp, &vits, &vrel, st);
  if (rc != SKIPM_OK) return fail_with(rc);
  rc = finish_step(lp, st);
  if (rc != SKIPM_OK) return fail_with(rc);
  lp->k += 1;
  b->it += 1;
}

void batch_cg_passes(skipm_lp_s* lp, ColPass normal[2], FinishDotArgs fin[2], ColPass close[2],
                     ColPass* qinit, CgInitArgs* init, CgCloseArgs* cls) {
  for (int p = 0; p < 2; ++p) {
    normal[p] = cg_normal_args(lp, p);
    fin[p] = cg_finish_args(lp, p, normal[p].nblk);
    close[p] = cg_close_args(lp, lp->dy, p);
  }
  ColPass q{};
  q.mode = COL_DOT;
  q.A = lp->G;
  q.ta = SKIPM_F64;
  q.tc = SKIPM_F64;
  q.lda = lp->mp;
  q.m = lp->mp;
  q.n = lp->m;
  q.u = lp->p;
  q.t_out = lp->cw;
  q.nblk = 0;
  *qinit = q;
  init->m = lp->m;
  init->rhs = lp->p;
  init->zin = lp->cw;
  init->r = lp->cr;
  init->z = lp->cz;
  init->d = lp->cd;
  init->x = lp->dy;
  init->sc = lp->sc;
  init->is = lp->is;
  init->tol = lp->prm.tol_cg;
  init->max_it = lp->prm.max_cg;
  cls->prz = lp->cgred + lp->cg_nf;
  cls->np = lp->cg_nd;
  cls->sc = lp->sc;
  cls->is = lp->is;
}

}  // namespace skipm

extern "C" {

int skipm_params_default(skipm_params* out) {
  if (!out) return set_error("null params"), SKIPM_EINVAL;
  memset(out, 0, sizeof(*out));
  out->sigma = 0.5;
  out->gamma = 0.999;
  out->tol_cg = 1e-5;
  out->eps_gap = 1e-6;
  out->eps_feas = 1e-8;
  out->guard = 1e-3;
  out->w = 0;
  out->s = 1;
  out->max_cg = 1000;
  out->max_outer = 300;
  out->resketch = 1;
  out->precision = SKIPM_PREC_FP64;
  out->seed = 0;
  out->inner = SKIPM_INNER_CG;
  out->sketch = SKIPM_SKETCH_COUNT;
  return SKIPM_OK;
}

int lp_footprint(const skipm_problem* prob, const skipm_params* prm, int64_t* out) {
  if (!prob || !prm || !out) return set_error("null argument"), SKIPM_EINVAL;
  const int64_t m = prob->m, n = prob->n;
  if (m < 1 || n < m || m > kMaxM) return set_error("need 1 <= m <= min(n, 2048)"), SKIPM_EINVAL;
  SK_TRY(validate_params(*prm, m, n));
  const bool csr = prob->format == SKIPM_CSR;
  const bool f64 = prob->a_dtype == SKIPM_F64;
  const int64_t esz = f64 ? 8 : 4;
  const int64_t lda = round_up(m, 4), mp = round_up(m, 64);
  const int64_t w = prm->w > 0 ? prm->w : 4 * m, s = prm->s;
  int64_t b = 0, nalloc = 0;
  auto add = [&](int64_t bytes) {
    b += std::max<int64_t>(bytes, 8);
    ++nalloc;
  };
  int nblk_csc = 0;
  if (!csr) {
    add(esz * lda * n);
    if (prm->precision != SKIPM_PREC_FP64 && f64) add(4 * lda * n);
    if (prm->precision == SKIPM_PREC_BF16) add(2 * round_up(m, 8) * n);
  } else {
    const int64_t nnz = prob->nnz;
    const int64_t nseg = m + nnz / kSeg + 1;
    add(4 * (m + 1));
    add(4 * nnz);
    add(4 * (n + 1));
    add(4 * nnz);
    add(4 * std::max(n, m));
    add(4 * std::max(n, m));
    add(4 * (m + 1));
    add(4 * m);
    add(4);
    add(8 * ((nnz * esz + 7) / 8));
    add(8 * ((nnz * esz + 7) / 8));
    add(4 * nseg);
    add(4 * nseg);
    add(8 * n);
    add(8 * n);
    add(16 * nseg);
    {  // column blocks: descriptors, the column-order copy, the row order
      // (FP64 values: a second keyed copy; FP32: 16-bit references)
      const int64_t nb = sb_max_blocks(n, nnz), sl = sb_max_slots(n, nnz);
      add(16 * nb);
      add(4 * sl);
      add(8 * ((sl * esz + 7) / 8));
      if (f64) {
        add(4 * sl);
        add(8 * ((sl * esz + 7) / 8));
      } else {
        add(8 * ((sl * 2 + 7) / 8));
      }
    }
    nblk_csc = csc_dot_nblk(n);
  }
  for (int i = 0; i < 8; ++i) add(8 * n);    // c x s d2 r_d dx ds v
  for (int i = 0; i < 19; ++i) add(8 * mp);  // m-vectors
  add(8 * (finish_nblk(m) +
           2 * (int64_t)colpass_nblk_dot(mp, m, SKIPM_F64)));  // CG partials
  add(8 * w);
  add(8 * w);
  add(8 * w);
  add(8 * lda * w);  // B
  add(8 * (int64_t)gram_ksplit(mp, w) * mp * mp);
  add(8 * mp * mp);
  add(8 * mp * mp);
  add(8 * mp * mp);  // scratch of the triangular inverse
  add(4 * n * s);
  add(n * s);
  add(4 * n * s);
  add(4 * n * s);
  add(4 * (w + 1));
  add(4 * w);
  add(4 * w);
  const int ta = prob->a_dtype;
  const int nblk_A = colpass_nblk(lda, n, ta, SKIPM_F64, COL_NORMAL);
  const int nblk_Ap = colpass_nblk(lda, n, ta, SKIPM_F64, COL_PROLOGUE);
  const int nblk_A32 = colpass_nblk(lda, n, SKIPM_F32, SKIPM_F64, COL_NORMAL);
  const int nblk_A16 = colpass_nblk(round_up(m, 8), n, kTypeBF16, SKIPM_F64, COL_NORMAL);
  const int nblk_B = colpass_nblk(lda, w, SKIPM_F64, SKIPM_F64, COL_NORMAL);
  const int nblk_vec = vec_nblk(n);
  int64_t pe = std::max<int64_t>(2 * (int64_t)nblk_Ap * mp, (int64_t)nblk_A * mp);
  pe = std::max<int64_t>(pe, (int64_t)nblk_B * mp);
  pe = std::max<int64_t>(pe, (int64_t)nblk_A32 * mp);
  pe = std::max<int64_t>(pe, (int64_t)nblk_A16 * mp);
  pe = std::max<int64_t>(pe, (int64_t)colpass_nblk(mp, m, SKIPM_F64, SKIPM_F64, COL_AXPY) * mp);
  if (csr) pe = std::max<int64_t>(pe, sb_max_blocks(n, prob->nnz) * mp);
  add(8 * pe);
  add(8 * 8 * (int64_t)std::max(std::max(std::max(nblk_Ap, nblk_vec), nblk_csc), 64));
  add(8 * S_NSLOTS);
  add(4 * I_NINTS);
  if (prm->sketch == SKIPM_SKETCH_GAUSSIAN) {  // D W_G, (D W_G) t, K-split slices
    add(8 * round_up(n, 2) * w);
    add(8 * n);
    const int ns = gauss_ksplit(lda, w, n);
    if (ns > 1) add(8 * ns * lda * w);
  }
  // correction-vector buffers (allocated at the first direction)
  add(8 * lda * w);
  add(8 * lda * w);
  for (int i = 0; i < 4; ++i) add(8 * mp * mp);
  // allocation granularity
  *out = b + nalloc * (int64_t)(64 << 10);
  return SKIPM_OK;
}

int lp_kernel_timing(skipm_lp_t lp, int32_t every) {
  if (!lp) return set_error("null handle"), SKIPM_EINVAL;
  if (every < 0) return set_error("every must be >= 0"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  if (every > 0 && lp->kt_ev.empty()) {
    lp->kt_ev.resize(2 * kKtPairs, nullptr);
    for (auto& e : lp->kt_ev) SK_CHECK_HIP(hipEventCreateWithFlags(&e, kTimingEvent));
  }
  if (every > 0 && !lp->ks_ev[0]) {
    SK_CHECK_HIP(hipEventCreateWithFlags(&lp->ks_ev[0], kTimingEvent));
    SK_CHECK_HIP(hipEventCreateWithFlags(&lp->ks_ev[1], kTimingEvent));
  }
  lp->kt_every = every;
  lp->kt_iter.clear();
  lp->kt_tier.clear();
  lp->kt_pair.clear();
  lp->kt_used = 0;
  lp->kt_sum_ms = 0;
  lp->kt_count = 0;
  for (int t = 0; t < 3; ++t) {
    lp->kt_tier_ms[t] = 0;
    lp->kt_tier_n[t] = 0;
  }
  lp->ks_pending = false;
  lp->ks_sum_ms = 0;
  lp->ks_count = 0;
  return SKIPM_OK;
}

int lp_sketch_time(skipm_lp_t lp, double* avg_ms, int64_t* samples) {
  if (!lp || !avg_ms || !samples) return set_error("null argument"), SKIPM_EINVAL;
  ks_harvest(lp);
  *samples = lp->ks_count;
  *avg_ms = lp->ks_count ? lp->ks_sum_ms / (double)lp->ks_count : 0.0;
  return SKIPM_OK;
}

int lp_kernel_time(skipm_lp_t lp, double* avg_ms, int64_t* samples) {
  if (!lp || !avg_ms || !samples) return set_error("null argument"), SKIPM_EINVAL;
  *samples = lp->kt_count;
  *avg_ms = lp->kt_count ? lp->kt_sum_ms / (double)lp->kt_count : 0.0;
  return SKIPM_OK;
}

int lp_kernel_time_tier(skipm_lp_t lp, int32_t tier, double* avg_ms, int64_t* samples) {
  if (!lp || !avg_ms || !samples) return set_error("null argument"), SKIPM_EINVAL;
  if (tier < SKIPM_TIER_FP64 || tier > SKIPM_TIER_BF16) return set_error("unknown tier"), SKIPM_EINVAL;
  *samples = lp->kt_tier_n[tier];
  *avg_ms = *samples ? lp->kt_tier_ms[tier] / (double)*samples : 0.0;
  return SKIPM_OK;
}

int lp_device_bytes(skipm_lp_t lp, int64_t* out) {
  if (!lp || !out) return set_error("null argument"), SKIPM_EINVAL;
  *out = lp->bytes;
  return SKIPM_OK;
}

int lp_destroy(skipm_lp_t lp) {
  if (!lp) return SKIPM_OK;
  // release everything; a failure here has nothing left to report to
  (void)hipSetDevice(lp->device);
  for (void* p : lp->allocs) (void)hipFree(p);
  for (hipEvent_t e : lp->kt_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : lp->ks_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : lp->snap_ev)
    if (e) (void)hipEventDestroy(e);
  if (lp->rd_ev) (void)hipEventDestroy(lp->rd_ev);
  for (double* h : {lp->hsc, lp->hsnap[0], lp->hsnap[1]})
    if (h) (void)hipHostFree(h);
  delete lp;
  return SKIPM_OK;
}

int lp_reset(skipm_lp_t lp, hipStream_t st) {
  if (!lp) return set_error("null handle"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  launch_fill_f64(lp->x, 1.0, lp->n, st);
  launch_fill_f64(lp->sv, 1.0, lp->n, st);
  launch_fill_f64(lp->y, 0.0, lp->mp, st);
  lp->k = 0;
  lp->prev_cg = 8;
  lp->last_rel_gap = HUGE_VAL;
  lp->origin_pending = 1;
  lp->small_steps = 0;
  lp->tier = lp->start_tier;
  lp->demote_iter = -1;
  lp->run_resketches = 0;
  lp->run_shifts = 0;
  SK_TRY(mu_from_iterate(lp, st));
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int lp_create(skipm_lp_t* out, const skipm_problem* prob, const skipm_params* prm,
              hipStream_t st) {
  if (!out || !prob || !prm) return set_error("null argument"), SKIPM_EINVAL;
  *out = nullptr;
  const int64_t m = prob->m, n = prob->n;
  if (m < 1 || n < m) return set_error("need 1 <= m <= n"), SKIPM_EINVAL;
  if (prob->format != SKIPM_DENSE && prob->format != SKIPM_CSR)
    return set_error("format must be SKIPM_DENSE or SKIPM_CSR"), SKIPM_EINVAL;
  if (prob->a_dtype != SKIPM_F64 && prob->a_dtype != SKIPM_F32)
    return set_error("a_dtype must be SKIPM_F64 or SKIPM_F32"), SKIPM_EINVAL;
  if (!prob->a_vals || !prob->b || !prob->c) return set_error("null problem pointer"), SKIPM_EINVAL;
  const bool csr = prob->format == SKIPM_CSR;
  if (csr && (!prob->a_rowptr || !prob->a_colidx))
    return set_error("CSR needs a_rowptr and a_colidx"), SKIPM_EINVAL;
  if (csr && (prob->nnz < 0 || prob->nnz > INT32_MAX))
    return set_error("nnz must lie in [0, 2^31)"), SKIPM_EINVAL;
  if (csr && n > INT32_MAX - 1) return set_error("n too large for int32 indices"), SKIPM_EINVAL;
  const int64_t lda_in = prob->lda > 0 ? prob->lda : m;
  if (!csr && lda_in < m) return set_error("lda < m"), SKIPM_EINVAL;
  SK_TRY(validate_params(*prm, m, n));
  if (m > kMaxM) return set_error("m <= 2048 is supported"), SKIPM_EINVAL;
  if (prm->sketch == SKIPM_SKETCH_GAUSSIAN && (csr || prob->a_dtype != SKIPM_F64))
    return set_error("the Gaussian sketch needs dense FP64 A"), SKIPM_EINVAL;

  skipm_lp_s* lp = new skipm_lp_s();
  if (hipGetDevice(&lp->device) != hipSuccess) {
    delete lp;
    return set_error("hipGetDevice failed"), SKIPM_EDEVICE;
  }
  lp->m = m;
  lp->n = n;
  lp->fmt = prob->format;
  lp->a_dtype = prob->a_dtype;
  lp->prm = *prm;
  lp->w = prm->w > 0 ? prm->w : (int)(4 * m);
  lp->s = prm->s;
  // a CSR problem's values are read as stored (FP32 or FP64) with FP64
  // accumulation in every pass, so it has no separate mixed mode
  lp->mixed = prm->precision != SKIPM_PREC_FP64 && !csr;
  const bool bf16 = prm->precision == SKIPM_PREC_BF16 && !csr;
  lp->start_tier = bf16 ? SKIPM_TIER_BF16 : (lp->mixed ? SKIPM_TIER_FP32 : SKIPM_TIER_FP64);
  lp->lda16 = round_up(m, 8);
  lp->tier = lp->start_tier;
  lp->lda = round_up(m, 4);
  lp->mp = round_up(m, 64);
  const int64_t mp = lp->mp, lda = lp->lda, w = lp->w;

  int rc = SKIPM_OK;
#define ALLOC(ptr, cnt)                      \
  if ((rc = dalloc(lp, &(ptr), (cnt))) != 0) { \
    lp_destroy(lp);                          \
    return rc;                               \
  }
  const size_t esz = lp->a_dtype == SKIPM_F64 ? 8 : 4;
  if (!csr) {
    void* p = nullptr;
    if (hipMalloc(&p, esz * lda * n) != hipSuccess) {
      lp_destroy(lp);
      return set_error("hipMalloc of A failed"), SKIPM_ENOMEM;
    }
    lp->allocs.push_back(p);
    lp->bytes += (int64_t)(esz * lda * n);
    lp->A = p;
  } else {
    const int64_t nnz = prob->nnz;
    lp->nnz = nnz;
    SparseA& S = lp->sp;
    S.m = m;
    S.n = n;
    S.nnz = nnz;
    S.vdt = lp->a_dtype;
    int32_t *rowptr, *colidx, *colptr, *rowidx, *cnt, *cursor, *segptr, *nsegv, *bad;
    void *val, *cval;
    ALLOC(rowptr, m + 1);
    ALLOC(colidx, nnz);
    ALLOC(colptr, n + 1);
    ALLOC(rowidx, nnz);
    ALLOC(cnt, std::max<int64_t>(n, m));
    ALLOC(cursor, std::max<int64_t>(n, m));
    ALLOC(segptr, m + 1);
    ALLOC(nsegv, m);
    ALLOC(bad, 1);
    {
      double* vp = nullptr;
      double* cp = nullptr;
      ALLOC(vp, (nnz * (int64_t)esz + 7) / 8);
      ALLOC(cp, (nnz * (int64_t)esz + 7) / 8);
      val = vp;
      cval = cp;
    }
    SK_CHECK_HIP(hipMemcpyAsync(rowptr, prob->a_rowptr, (m + 1) * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, st));
    if (nnz > 0) {
      SK_CHECK_HIP(hipMemcpyAsync(colidx, prob->a_colidx, nnz * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, st));
      SK_CHECK_HIP(hipMemcpyAsync(val, prob->a_vals, nnz * esz, hipMemcpyDeviceToDevice, st));
    }
    launch_fill_i32(bad, 0, 1, st);
    launch_csr_check(rowptr, colidx, m, n, nnz, bad, st);
    int32_t hbad = 0;
    SK_CHECK_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SK_CHECK_HIP(hipStreamSynchronize(st));
    if (hbad) {
      lp_destroy(lp);
      return set_error(hbad & 1 ? "CSR row pointers are invalid"
                                : "CSR column indices out of range or not increasing"),
             SKIPM_EINVAL;
    }
    launch_build_csc(rowptr, colidx, val, lp->a_dtype, m, n, nnz, cnt, colptr, cursor, rowidx,
                     cval, st);
    launch_build_segments(rowptr, m, kSeg, nsegv, segptr, cursor, nullptr, nullptr, st);
    int32_t hnseg = 0;
    SK_CHECK_HIP(hipMemcpyAsync(&hnseg, segptr + m, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SK_CHECK_HIP(hipStreamSynchronize(st));
    int32_t *seg_start, *seg_end;
    ALLOC(seg_start, hnseg);
    ALLOC(seg_end, hnseg);
    launch_build_segments(rowptr, m, kSeg, nsegv, segptr, cursor, seg_start, seg_end, st);
    S.rowptr = rowptr;
    S.colidx = colidx;
    S.val = val;
    S.colptr = colptr;
    S.rowidx = rowidx;
    S.cval = cval;
    S.nseg = hnseg;
    S.segptr = segptr;
    S.seg_start = seg_start;
    S.seg_end = seg_end;
    ALLOC(lp->cf1, n);
    ALLOC(lp->cf2, n);
    ALLOC(lp->segsum, 2 * (int64_t)hnseg);
    lp->nblk_csc = csc_dot_nblk(n);
    // column blocks of the one-pass normal product
    {
      std::vector<int32_t> hd;
      const int64_t slots = sb_partition(S, &hd, st);
      const int64_t nbk = (int64_t)hd.size() / 4;
      if (slots < 0 || nbk < 1 || nbk > sb_max_blocks(n, nnz) || slots > sb_max_slots(n, nnz)) {
        lp_destroy(lp);
        return set_error("sparse block partition failed"), SKIPM_EDEVICE;
      }
      S.nbk = nbk;
      int32_t* bdesc;
      uint32_t* ck;
      uint32_t* rk = nullptr;
      double* cv;
      double* rv = nullptr;
      uint16_t* rp = nullptr;
      ALLOC(bdesc, 4 * nbk);
      ALLOC(ck, slots);
      ALLOC(cv, (slots * (int64_t)esz + 7) / 8);
      if (S.vdt == SKIPM_F64) {
        ALLOC(rk, slots);
        ALLOC(rv, (slots * (int64_t)esz + 7) / 8);
      } else {
        ALLOC(rp, slots);
      }
      SK_CHECK_HIP(hipMemcpyAsync(bdesc, hd.data(), 4 * nbk * sizeof(int32_t),
                                  hipMemcpyHostToDevice, st));
      sb_fill(&S, bdesc, ck, cv, rk, rv, rp, bad, st);
      SK_CHECK_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      SK_CHECK_HIP(hipStreamSynchronize(st));
      if (hbad) {
        lp_destroy(lp);
        return set_error("sparse block exceeds its bounds"), SKIPM_EDEVICE;
      }
    }
  }
  if (lp->mixed && lp->a_dtype == SKIPM_F64) ALLOC(lp->A32, lda * n);
  if (bf16) ALLOC(lp->A16, lp->lda16 * n);
  ALLOC(lp->b, mp);
  ALLOC(lp->c, n);
  ALLOC(lp->x, n);
  ALLOC(lp->y, mp);
  ALLOC(lp->sv, n);
  ALLOC(lp->d2, n);
  ALLOC(lp->rd, n);
  ALLOC(lp->dx, n);
  ALLOC(lp->ds, n);
  ALLOC(lp->v, n);
  ALLOC(lp->rp, mp);
  ALLOC(lp->p, mp);
  ALLOC(lp->dy, mp);
  ALLOC(lp->g, mp);
  ALLOC(lp->cr, mp);
  ALLOC(lp->cz, mp);
  ALLOC(lp->cd, mp);
  ALLOC(lp->cd2, mp);
  lp->cg_nf = finish_nblk(m);
  {
    // one-workgroup CG for small dense LPs; SKIPM_CG_SMALL_BYTES overrides the
    // size limit of A's CG copy (0 turns it off)
    lp->small_cg_bytes = 1 << 20;
    if (const char* e = getenv("SKIPM_CG_SMALL_BYTES")) lp->small_cg_bytes = atoll(e);
    // SKIPM_STEP_ONE=0 keeps the multi-launch step tail for every n (the
    // one-workgroup tail computes the same sums in the same order)
    if (const char* e = getenv("SKIPM_STEP_ONE")) lp->step_one = atoi(e) != 0;
  }
  lp->cg_nd = colpass_nblk_dot(mp, m, SKIPM_F64);
  ALLOC(lp->cgred, lp->cg_nf + 2 * (int64_t)lp->cg_nd);
  ALLOC(lp->cq, mp);
  ALLOC(lp->cw, mp);
  ALLOC(lp->cx, mp);
  ALLOC(lp->rv, mp);
  ALLOC(lp->rv2, mp);
  ALLOC(lp->rt, mp);
  ALLOC(lp->dyc, mp);
  ALLOC(lp->uv1, mp);
  ALLOC(lp->uv2, mp);
  ALLOC(lp->tw, w);
  ALLOC(lp->tw2, w);
  ALLOC(lp->tq, w);
  ALLOC(lp->B, lda * w);
  lp->ksplit = gram_ksplit(mp, w);
  ALLOC(lp->Gpart, (int64_t)lp->ksplit * mp * mp);
  ALLOC(lp->G, mp * mp);
  ALLOC(lp->Xb, mp * mp);
  ALLOC(lp->Ct, mp * mp);
  ALLOC(lp->bucket, n * lp->s);
  ALLOC(lp->sign, n * lp->s);
  ALLOC(lp->perm, n * lp->s);
  ALLOC(lp->perm_raw, n * lp->s);
  ALLOC(lp->bptr, w + 1);
  ALLOC(lp->bcnt, w);
  ALLOC(lp->bcur, w);
  lp->nblk_A = colpass_nblk(lda, n, lp->a_dtype, SKIPM_F64, COL_NORMAL);
  lp->nblk_Ap = colpass_nblk(lda, n, lp->a_dtype, SKIPM_F64, COL_PROLOGUE);
  lp->nblk_A32 = colpass_nblk(lda, n, SKIPM_F32, SKIPM_F64, COL_NORMAL);
  lp->nblk_A16 = colpass_nblk(lp->lda16, n, kTypeBF16, SKIPM_F64, COL_NORMAL);
  lp->nblk_B = colpass_nblk(lda, w, SKIPM_F64, SKIPM_F64, COL_NORMAL);
  lp->nblk_vec = vec_nblk(n);
  {
    int64_t pe = std::max<int64_t>(2 * (int64_t)lp->nblk_Ap * mp, (int64_t)lp->nblk_A * mp);
    pe = std::max<int64_t>(pe, (int64_t)lp->nblk_B * mp);
    pe = std::max<int64_t>(pe, (int64_t)lp->nblk_A32 * mp);
    pe = std::max<int64_t>(pe, (int64_t)lp->nblk_A16 * mp);
    pe = std::max<int64_t>(pe, (int64_t)colpass_nblk(mp, m, SKIPM_F64, SKIPM_F64, COL_AXPY) * mp);
    if (csr) pe = std::max<int64_t>(pe, lp->sp.nbk * mp);
    ALLOC(lp->part, pe);
  }
  ALLOC(lp->red,
        (int64_t)std::max(std::max(std::max(lp->nblk_Ap, lp->nblk_vec), lp->nblk_csc), 64) * 8);
  // the FP64 slots and the int32 slots in one allocation, laid out as the
  // host mirror hsc, so a host read is one copy
  ALLOC(lp->sc, S_NSLOTS + (I_NINTS + 1) / 2);
  lp->is = (int32_t*)(lp->sc + S_NSLOTS);
#undef ALLOC
  for (double** h : {&lp->hsc, &lp->hsnap[0], &lp->hsnap[1]}) {
    if (hipHostMalloc((void**)h, kScalarBlockBytes) != hipSuccess) {
      lp_destroy(lp);
      return set_error("hipHostMalloc failed"), SKIPM_ENOMEM;
    }
  }
  for (hipEvent_t* e : {&lp->snap_ev[0], &lp->snap_ev[1], &lp->rd_ev}) {
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      lp_destroy(lp);
      return set_error("hipEventCreate failed"), SKIPM_EDEVICE;
    }
  }
  // zero the vectors whose padding must stay zero, then copy the problem in
  launch_fill_f64(lp->sc, 0.0, S_NSLOTS, st);
  launch_fill_i32(lp->is, 0, I_NINTS, st);
  double* zero_vecs[] = {lp->b,  lp->y,  lp->rp, lp->p,  lp->dy, lp->g,  lp->cr,  lp->cz,
                         lp->cd, lp->cd2, lp->cq, lp->cw, lp->cx, lp->rv, lp->rv2, lp->uv1,
                         lp->uv2, lp->rt, lp->dyc};
  for (double* z : zero_vecs) launch_fill_f64(z, 0.0, mp, st);
  launch_fill_f64(lp->B, 0.0, lda * w, st);
  launch_copy_f64(lp->b, prob->b, m, st);
  launch_copy_f64(lp->c, prob->c, n, st);
  if (csr) {
    // A lives in lp->sp
  } else if (lp->a_dtype == SKIPM_F64) {
    launch_pad_copy_f64((double*)lp->A, lda, (const double*)prob->a_vals, lda_in, m, n, st);
    if (lp->mixed)
      launch_pad_copy_f64_to_f32(lp->A32, lda, (const double*)prob->a_vals, lda_in, m, n, st);
  } else {
    launch_pad_copy_f32((float*)lp->A, lda, (const float*)prob->a_vals, lda_in, m, n, st);
    if (lp->mixed) lp->A32 = (float*)lp->A;
  }
  if (bf16)
    launch_pad_copy_to_bf16(lp->A16, lp->lda16, prob->a_vals, lp->a_dtype, lda_in, m, n, st);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    lp_destroy(lp);
    return set_error("device error while copying the problem"), SKIPM_EDEVICE;
  }
  if ((rc = set_param_slots(lp, st)) != SKIPM_OK || (rc = lp_reset(lp, st)) != SKIPM_OK) {
    lp_destroy(lp);
    return rc;
  }
  lp->bnorm = host_norm(lp->b, m, &rc);
  if (rc == SKIPM_OK) lp->cnorm = host_norm(lp->c, n, &rc);
  if (rc != SKIPM_OK) {
    lp_destroy(lp);
    return set_error("copy of b or c failed"), rc;
  }
  *out = lp;
  return SKIPM_OK;
}

int lp_set_iterate(skipm_lp_t lp, const double* x, const double* y, const double* s,
                   int32_t reset_origin, hipStream_t st) {
  if (!lp || !x || !y || !s) return set_error("null argument"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  launch_copy_f64(lp->x, x, lp->n, st);
  launch_copy_f64(lp->y, y, lp->m, st);
  launch_copy_f64(lp->sv, s, lp->n, st);
  lp->last_rel_gap = HUGE_VAL;
  if (reset_origin) {
    lp->origin_pending = 1;
    lp->k = 0;
  }
  SK_TRY(mu_from_iterate(lp, st));
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int lp_get_iterate(skipm_lp_t lp, double* x, double* y, double* s, hipStream_t st) {
  if (!lp) return set_error("null handle"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  if (x) launch_copy_f64(x, lp->x, lp->n, st);
  if (y) launch_copy_f64(y, lp->y, lp->m, st);
  if (s) launch_copy_f64(s, lp->sv, lp->n, st);
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int lp_get_direction(skipm_lp_t lp, double* dx, double* dy, double* ds, double* v,
                     hipStream_t st) {
  if (!lp) return set_error("null handle"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  if (dx) launch_copy_f64(dx, lp->dx, lp->n, st);
  if (dy) launch_copy_f64(dy, lp->dy, lp->m, st);
  if (ds) launch_copy_f64(ds, lp->ds, lp->n, st);
  if (v) launch_copy_f64(v, lp->v, lp->n, st);
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int lp_get_residuals(skipm_lp_t lp, double* rp, double* rd, double* p, double* g,
                     hipStream_t st) {
  if (!lp) return set_error("null handle"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  if (rp) launch_copy_f64(rp, lp->rp, lp->m, st);
  if (rd) launch_copy_f64(rd, lp->rd, lp->n, st);
  if (p) launch_copy_f64(p, lp->p, lp->m, st);
  if (g) launch_copy_f64(g, lp->g, lp->m, st);
  SK_CHECK_HIP(hipGetLastError());
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int sketch_hash(uint64_t seed, int64_t k, int32_t s, int64_t n, int32_t w, int32_t* bucket,
                int8_t* sign, hipStream_t st) {
  if (!bucket || !sign) return set_error("null output"), SKIPM_EINVAL;
  if (n < 1 || w < 1 || s < 1 || s > 16 || w % s != 0)
    return set_error("need n >= 1, 1 <= s <= 16, s | w"), SKIPM_EINVAL;
  launch_hash(seed, k, s, n, w, bucket, sign, nullptr, st);
  SK_CHECK_HIP(hipGetLastError());
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int sketch_apply(skipm_lp_t lp, const double* d, int64_t k, void* B, int32_t out_dtype,
                 hipStream_t st) {
  if (out_dtype != SKIPM_F64 && out_dtype != SKIPM_F32)
    return set_error("out_dtype must be SKIPM_F64 or SKIPM_F32"), SKIPM_EINVAL;
  if (!lp || !d || !B) return set_error("null argument"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  SK_TRY(sketch_into(lp, d, 0, k, lp->B, st));
  if (out_dtype == SKIPM_F64)
    launch_pad_copy_f64((double*)B, lp->m, lp->B, lp->lda, lp->m, lp->w, st);
  else
    launch_pad_copy_f64_to_f32((float*)B, lp->m, lp->B, lp->lda, lp->m, lp->w, st);
  SK_CHECK_HIP(hipGetLastError());
  SK_CHECK_HIP(hipStreamSynchronize(st));
  return SKIPM_OK;
}

int pcg_solve(skipm_lp_t lp, const double* d2, const double* p, int64_t k, double* dy, double tol,
              int32_t max_it, skipm_pcg_info* info, hipStream_t st) {
  if (!lp || !d2 || !p || !dy) return set_error("null argument"), SKIPM_EINVAL;
  if (max_it < 1) return set_error("max_it must be >= 1"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  launch_copy_f64(lp->d2, d2, lp->n, st);
  launch_copy_f64(lp->g, p, lp->m, st);  // g doubles as the right-hand side buffer here
  int its = 0;
  SK_TRY(sketch_solve(lp, lp->d2, 1, k, lp->g, lp->cx, tol, max_it, &its, st));
  launch_copy_f64(dy, lp->cx, lp->m, st);
  SK_CHECK_HIP(hipGetLastError());
  SK_CHECK_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iters = its;
    info->f0_norm = sqrt(std::max(0.0, lp->hsc[S_CG_RZ0]));
    info->f_norm = sqrt(std::max(0.0, lp->hsc[S_CG_RZ]));
  }
  return SKIPM_OK;
}

static int normal_matvec_impl(skipm_lp_t lp, const double* u, double* out, int32_t reps,
                              float* ms, hipStream_t st);

int normal_matvec(skipm_lp_t lp, const double* u, double* out, int32_t reps, hipStream_t st) {
  return normal_matvec_impl(lp, u, out, reps, nullptr, st);
}

int normal_matvec_timed(skipm_lp_t lp, const double* u, double* out, int32_t reps,
                        float* ms_per_pass, hipStream_t st) {
  if (!ms_per_pass) return set_error("null ms_per_pass"), SKIPM_EINVAL;
  return normal_matvec_impl(lp, u, out, reps, ms_per_pass, st);
}

static int normal_matvec_impl(skipm_lp_t lp, const double* u, double* out, int32_t reps,
                              float* ms, hipStream_t st) {
  if (!lp || !u || !out) return set_error("null argument"), SKIPM_EINVAL;
  if (reps < 1) return set_error("reps must be >= 1"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  launch_copy_f64(lp->cd, u, lp->m, st);
  if (lp->fmt == SKIPM_CSR) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
      SK_CHECK_HIP(hipEventCreateWithFlags(&e0, kTimingEvent));
      SK_CHECK_HIP(hipEventCreateWithFlags(&e1, kTimingEvent));
      SK_CHECK_HIP(hipEventRecord(e0, st));
    }
    for (int r = 0; r < reps; ++r) SK_TRY(normal_sparse(lp, lp->cd, 1.0, nullptr, 0.0, out, nullptr, st));
    if (ms) {
      float tot = 0;
      SK_CHECK_HIP(hipEventRecord(e1, st));
      SK_CHECK_HIP(hipEventSynchronize(e1));
      SK_CHECK_HIP(hipEventElapsedTime(&tot, e0, e1));
      *ms = tot / (float)reps;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    SK_CHECK_HIP(hipGetLastError());
    return SKIPM_OK;
  }
  ColPass cp = colpass_A(lp, COL_NORMAL);
  cp.u = lp->cd;
  cp.d2 = lp->d2;
  use_tier_copy(lp, cp);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    SK_CHECK_HIP(hipEventCreateWithFlags(&e0, kTimingEvent));
    SK_CHECK_HIP(hipEventCreateWithFlags(&e1, kTimingEvent));
    SK_CHECK_HIP(hipEventRecord(e0, st));
  }
  for (int r = 0; r < reps; ++r) SK_TRY(run_colpass(cp, st));
  if (ms) SK_CHECK_HIP(hipEventRecord(e1, st));
  launch_finish(lp->part, lp->mp, 0, cp.nblk, lp->m, 1.0, nullptr, 0.0, out, nullptr, st);
  SK_CHECK_HIP(hipGetLastError());
  if (ms) {
    float tot = 0;
    SK_CHECK_HIP(hipEventSynchronize(e1));
    SK_CHECK_HIP(hipEventElapsedTime(&tot, e0, e1));
    *ms = tot / (float)reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return SKIPM_OK;
}

int ipm_step(skipm_lp_t lp, skipm_step_info* info, hipStream_t st) {
  if (!lp) return set_error("null handle"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  const double bn = lp->bnorm, cn = lp->cnorm;
  const int rc = step_internal(lp, info, bn, cn, st);
  if (rc != SKIPM_OK) return rc;
  if (info && !info->converged) {
    SK_TRY(sync_read(lp, st));
    info->alpha_max = lp->hsc[S_AMAX];
    info->alpha = lp->hsc[S_ALPHA];
    info->v_norm = sqrt(std::max(0.0, lp->hsc[S_V2]));
  }
  return SKIPM_OK;
}

int lp_solve(skipm_lp_t lp, skipm_result* res, hipStream_t st) {
  if (!lp || !res) return set_error("null argument"), SKIPM_EINVAL;
  SK_CHECK_HIP(hipSetDevice(lp->device));
  const double bn = lp->bnorm, cn = lp->cnorm;
  memset(res, 0, sizeof(*res));
  int status = SKIPM_ENOTCONV;
  int it = 0;
  for (;; ++it) {
    skipm_step_info info;
    if (it >= lp->prm.max_outer) {
      // evaluate the stopping test at the final iterate without stepping
      SK_TRY(prologue(lp, st));
      SK_TRY(sync_read(lp, st));
      const StopState ss = stop_test(lp, bn, cn);
      status = ss.converged ? SKIPM_OK : (ss.nan ? SKIPM_ENAN : SKIPM_ENOTCONV);
      break;
    }
    const int rc = step_internal(lp, &info, bn, cn, st);
    if (rc != SKIPM_OK) {
      status = rc;
      break;
    }
    if (info.converged) {
      status = SKIPM_OK;
      break;
    }
    res->cg_total += info.cg_iters;
    res->cg_max = std::max(res->cg_max, info.cg_iters);
  }
  fill_result(lp, res, status, it);
  if (status != SKIPM_OK && status != SKIPM_ENOTCONV) return status;
  return status == SKIPM_ENOTCONV ? (set_error("max_outer reached"), SKIPM_ENOTCONV) : SKIPM_OK;
}

const char* skipm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
