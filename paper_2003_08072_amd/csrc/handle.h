// The solver handle (skipm_lp_s) and the internal steps of one IPM
// iteration, shared by the single-LP entry points (api.hip) and the grouped
// batch engine (grouped.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <string>
#include <vector>

#include "common.h"

struct skipm_lp_s {
  int device = 0;
  int64_t bytes = 0;  // device bytes held (every allocation of the handle)
  int64_t m = 0, n = 0, nnz = 0;
  int fmt = SKIPM_DENSE, a_dtype = SKIPM_F64;
  int64_t lda = 0, mp = 0;
  skipm_params prm{};
  int w = 0, s = 1;
  bool mixed = false;
  // device buffers
  void* A = nullptr;
  float* A32 = nullptr;
  uint16_t* A16 = nullptr;  // bfloat16 copy of A (precision SKIPM_PREC_BF16)
  int64_t lda16 = 0;        // its leading dimension: m rounded up to 8 (16-byte columns)
  double *b = nullptr, *c = nullptr, *x = nullptr, *y = nullptr, *sv = nullptr;
  double *d2 = nullptr, *rd = nullptr, *dx = nullptr, *ds = nullptr, *v = nullptr;
  double *rp = nullptr, *p = nullptr, *dy = nullptr, *g = nullptr;
  double *cr = nullptr, *cz = nullptr, *cd = nullptr, *cq = nullptr, *cw = nullptr,
         *cx = nullptr;
  double *tw = nullptr, *tq = nullptr;
  double* B = nullptr;
  double* Gpart = nullptr;
  int ksplit = 1;
  double* G = nullptr;
  double* Xb = nullptr;
  // correction-vector solve: whitened sketches B1 = L0^{-1} B, B2 = L1^{-1} B1, their
  // Gram inverses, and the accumulated inverse factors M1 = X0, M2 = X1 X0
  double *B1 = nullptr, *B2 = nullptr, *Gv = nullptr, *Xv = nullptr, *M1 = nullptr,
         *M2 = nullptr, *rv = nullptr, *uv1 = nullptr, *uv2 = nullptr;
  double *rt = nullptr, *dyc = nullptr;  // mixed precision: FP64 residual and correction
  // correction vector: the best t so far and its residual (tw, rv), and the
  // candidate of the current refinement step (tw2, rv2)
  double *tw2 = nullptr, *rv2 = nullptr;
  int last_outer = 0;
  // precision tier of the CG products (SKIPM_TIER_*): start_tier from the
  // parameters, tier the current one (it only moves up within a run)
  int start_tier = SKIPM_TIER_FP64, tier = SKIPM_TIER_FP64;
  int demote_iter = -1;  // IPM iteration of the first move up, -1 if none
  // rank-loss handling of the current solve and of the run (Lemma 3)
  int step_resketches = 0, step_shifts = 0;
  int run_resketches = 0, run_shifts = 0;
  int vrounds_built = 0;
  // CSR storage (format SKIPM_CSR)
  skipm::SparseA sp;
  double *cf1 = nullptr, *cf2 = nullptr, *segsum = nullptr;
  int nblk_csc = 1;
  int32_t *bucket = nullptr, *perm = nullptr, *perm_raw = nullptr, *bptr = nullptr,
          *bcnt = nullptr, *bcur = nullptr;
  int8_t* sign = nullptr;
  double* part = nullptr;  // column-pass partial sums
  double* red = nullptr;
  double* sc = nullptr;
  int32_t* is = nullptr;
  double* hsc = nullptr;  // pinned: S_NSLOTS doubles then I_NINTS ints
  // two more pinned copies of the scalar block, filled alternately by the CG's
  // chunk checks (the host reads one while the next chunk runs)
  double* hsnap[2] = {nullptr, nullptr};
  hipEvent_t snap_ev[2] = {nullptr, nullptr};
  hipEvent_t rd_ev = nullptr;  // marks the end of a synchronous read of the scalar block
  // false: each chunk is checked with the stream idle (no chunk queued behind
  // the check); set for LPs that the batch and the request server solve on
  // their own threads, where other LPs keep the device busy meanwhile
  bool overlap_checks = true;
  int nblk_A = 1, nblk_Ap = 1, nblk_A32 = 1, nblk_A16 = 1, nblk_B = 1, nblk_vec = 1;
  int64_t k = 0;
  int64_t hashed_k = -1;
  int prev_cg = 8;
  double last_rel_gap = HUGE_VAL;  // relative gap at the last stopping test
  int origin_pending = 1;
  int small_steps = 0;
  double bnorm = 0, cnorm = 0;
  // fused CG (dense A): second direction buffer and the partial sums
  double* cd2 = nullptr;
  double* Ct = nullptr;  // mp x mp scratch of the triangular inverse
  // Gaussian sketch: Wd = D W_G (n x w, leading dimension ldw = n rounded up
  // to even, so its columns are 16-byte aligned), (D W_G) t for the correction
  // vector
  double* Wd = nullptr;
  int64_t ldw = 0;
  double* gy = nullptr;
  double* Bsplit = nullptr;  // K-split partial sketches of the Gaussian GEMM
  double* cgred = nullptr;  // [cg_nf] d^T q partials, then [cg_nd][2] r^T z, r^T r partials
  int cg_nf = 0, cg_nd = 0;
  int64_t small_cg_bytes = 0;  // dense CG in one workgroup when A's CG copy is at most this
  int step_one = 1;  // one-workgroup step tail where the n-vector passes take one workgroup
  std::vector<void*> allocs;
  // sampled HIP-event timing of the CG's normal-equation product (lp_kernel_timing):
  // event pairs around every kt_every-th product, harvested at the CG's host checks
  int kt_every = 0;
  std::vector<hipEvent_t> kt_ev;  // 2 * kKtPairs events
  std::vector<int> kt_iter;       // CG iteration of each pending sample
  std::vector<int> kt_tier;       // precision tier of the product it brackets
  std::vector<int> kt_pair;       // its event pair
  uint64_t kt_used = 0;           // event pairs held by pending samples (bit per pair)
  double kt_sum_ms = 0;
  int64_t kt_count = 0;
  double kt_tier_ms[3] = {0, 0, 0};  // the same, per SKIPM_TIER_*
  int64_t kt_tier_n[3] = {0, 0, 0};
  // event pair around the sketch product of every IPM iteration while timing is on
  hipEvent_t ks_ev[2] = {nullptr, nullptr};
  bool ks_pending = false;
  double ks_sum_ms = 0;
  int64_t ks_count = 0;
};

namespace skipm {

// Wait for ev (recorded on the awaited stream): polled for a while, then a
// blocking wait.  wait_stream records ev on st first (a plain stream
// synchronisation when ev is null).
int poll_event(hipEvent_t ev);
int wait_stream(hipStream_t st, hipEvent_t ev);

// ---- one IPM iteration in steps, for the grouped batch engine ----------------
// Each step is exactly what lp_solve does at that point of an iteration, so an
// LP driven through them takes the same arithmetic as a lone solve.

// Per-LP state of a batch run (the loop variables of lp_solve).
struct BatchLp {
  int it = 0;          // IPM iterations taken
  bool active = true;  // false once the run has ended (res->status holds why)
  bool grouped = false;  // this iteration's CG runs in the grouped launches
  int its = 0;         // CG iterations of this iteration
  int fail = 0;        // the factorisation met a non-positive pivot
  int rc = SKIPM_OK;   // an argument, memory or device error (ends the batch)
  std::string err;     // its message (errors are per thread)
};

// The LPs the grouped engine drives: dense, FP64 products (tier FP64 from the
// start).  Their CG runs in the grouped launches unless it runs in one
// workgroup (small dense FP64 LPs), as a lone solve would take it.
bool batch_groupable(const skipm_lp_s* lp);
// Start of an iteration: stopping test (ends the run if it holds or the run
// failed), then the sketch and the Gram factorisation; an LP whose CG runs in
// one workgroup also runs its CG here.
void batch_phase_a(skipm_lp_s* lp, skipm_result* res, BatchLp* b, hipStream_t st);
// End of an iteration, after the CG: the rank-loss retries if the
// factorisation failed, the epilogue, the correction vector, the step.
void batch_phase_b(skipm_lp_s* lp, skipm_result* res, BatchLp* b, hipStream_t st);
// The CG passes of this LP as the lone CG launches them: the product pass
// (normal[p]), the finish (fin[p]) and the Q^{-1} pass (close[p]) of
// iterations of parity p; the Q^{-1} application that starts the CG (qinit);
// the CG set-up and cap-closing arguments.
void batch_cg_passes(skipm_lp_s* lp, ColPass normal[2], FinishDotArgs fin[2], ColPass close[2],
                     ColPass* qinit, CgInitArgs* init, CgCloseArgs* cls);

}  // namespace skipm
