// The sparse normal product q = A diag(c) A^T u in one pass over column blocks.
//
// A's columns are cut into blocks of consecutive columns (at most kSbCols
// columns and kSbEntries non-zeros each).  Each block's non-zeros are kept
// once more in column order (ck = local column << 16 | row, cv: the value),
// and their (row, column) order is kept as well: with FP64 values as a second
// keyed copy (rk = row << 16 | local column, rv: the value), with FP32 values
// as 16-bit references to the column-order entries (rp, 2 bytes instead of
// 8 per non-zero; the workgroup reads the entries back from LDS).  Each key
// (reference) also marks the first and last non-zero of its column (row).
// In each order thread t of the block's workgroup (1024 threads) owns the
// K = ceil(N / 1024) consecutive non-zeros t K ... t K + K - 1 of the order,
// stored so that the k-th of them sits at slot k * 1024 + t of the block's
// region: a load of slot row k by all threads is coalesced, and each thread
// still walks a contiguous run.  One workgroup per block:
//   1. u (or, when the pass opens a CG iteration, d_k = z_k + beta_k d_{k-1})
//      into LDS, and all of the block's keys and values into registers (FP32:
//      the column-order entries also into LDS, by block-local slot);
//   2. column phase: each thread sums a_ij u_i along its run; columns inside
//      the run are complete, columns cut by run boundaries are joined by one
//      segmented scan over the threads; coef_j = c_j t_j into LDS;
//   3. row phase: the same over the row order with terms a_ij coef_j, giving
//      the block's q in LDS;
//   4. q goes to part[block]; the finish adds the partials of all blocks in
//      block order.
// coef never leaves LDS, so no value is gathered from global memory at a random
// column, no floating-point atomics are used, and the order of every addition
// is fixed by the data: results are bitwise reproducible.
#include <vector>

#include "common.h"

namespace skipm {

namespace {

constexpr int kSbThreads = 1024;
constexpr int kSbCols = 4096;      // columns per block (coefficients in LDS)
constexpr int kSbEntries = 8192;   // non-zeros per block
constexpr int kSbK = kSbEntries / kSbThreads;  // most non-zeros per thread
constexpr int kSbCap = kSbEntries - (int)kMaxM;  // see sb_partition
constexpr int kSbRows = (int)kMaxM;
constexpr uint32_t kSbFirst = 1u << 12, kSbLast = 1u << 13;  // key flags
constexpr uint32_t kSbLow = 0xfffu;  // local column (rk) or row (ck) bits
// row-order references (FP32 values): block-local slot, row's first / last
constexpr uint16_t kRpSlot = 0x1fff, kRpFirst = 1u << 13, kRpLast = 1u << 14;
template <typename TV>
constexpr bool sb_refs() { return sizeof(TV) == 4; }

__host__ __device__ inline int sb_k(int64_t N) { return (int)((N + kSbThreads - 1) / kSbThreads); }

// LDS slot of coefficient lc: one pad double after every eight, so that lanes
// reading or writing coefficients 4 or 8 apart (a thread's run over short
// columns, or over one long row) fall in different banks
__device__ __forceinline__ int cpad(int lc) { return lc + (lc >> 3); }
constexpr int kSbCoefLds = kSbCols + kSbCols / 8;

// One workgroup per block.  Column order: the CSC order.  Row order: the
// non-zeros keyed (row << 16 | local column) << 32 | CSC offset, bitonic-sorted
// in LDS (keys are distinct).  Logical position j of an order goes to slot
// (j % K) * 1024 + j / K of the block's region; a reference (FP32 values)
// names the block-local slot of the entry's column-order position.
template <typename TV>
__global__ __launch_bounds__(1024) void k_sb_sort(const int32_t* __restrict__ colptr,
                                                  const int32_t* __restrict__ rowidx,
                                                  const TV* __restrict__ cval,
                                                  const int4* __restrict__ bdesc,
                                                  uint32_t* __restrict__ ck, TV* __restrict__ cv,
                                                  uint32_t* __restrict__ rk, TV* __restrict__ rv,
                                                  uint16_t* __restrict__ rp,
                                                  int32_t* __restrict__ bad) {
  __shared__ uint64_t sk[kSbEntries];
  const int4 bd = bdesc[blockIdx.x];  // first column, columns, non-zeros, first slot
  const int64_t c0 = bd.x, c1 = (int64_t)bd.x + bd.y;
  const int64_t P0 = colptr[c0], P1 = colptr[c1];
  const int64_t O = bd.w;
  const int N = (int)(P1 - P0);
  if (N != bd.z || N > kSbEntries || bd.y > kSbCols) {
    if (threadIdx.x == 0) atomicOr(bad, 4);  // cannot happen by sb_partition's rule
    return;
  }
  const int K = sb_k(N);
  auto slot = [&](int j) { return O + (int64_t)(j % K) * kSbThreads + j / K; };
  int NP = 1;
  while (NP < N) NP <<= 1;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const int64_t pb = colptr[c], pe = colptr[c + 1];
    const uint32_t lc = (uint32_t)(c - c0);
    for (int64_t p = pb; p < pe; ++p) {
      const uint32_t r = (uint32_t)rowidx[p];
      const int j = (int)(p - P0);
      ck[slot(j)] = (lc << 16) | r | (p == pb ? kSbFirst : 0u) | (p == pe - 1 ? kSbLast : 0u);
      cv[slot(j)] = cval[p];
      sk[j] = ((uint64_t)((r << 16) | lc) << 32) | (uint64_t)j;
    }
  }
  for (int q = N + threadIdx.x; q < NP; q += blockDim.x) sk[q] = ~0ull;
  __syncthreads();
  for (int size = 2; size <= NP; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = threadIdx.x; q < NP / 2; q += blockDim.x) {
        const int lo = 2 * q - (q & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = sk[lo], y = sk[hi];
        if ((x > y) == up) {
          sk[lo] = y;
          sk[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    const uint64_t v = sk[q];
    const uint32_t key = (uint32_t)(v >> 32);
    const uint32_t row = key >> 16;
    const bool first = q == 0 || (uint32_t)(sk[q - 1] >> 48) != row;
    const bool last = q == N - 1 || (uint32_t)(sk[q + 1] >> 48) != row;
    const int jc = (int)(v & 0xffffffffull);
    if constexpr (sb_refs<TV>()) {
      rp[slot(q)] = (uint16_t)(((jc % K) * kSbThreads + jc / K) | (first ? kRpFirst : 0) |
                               (last ? kRpLast : 0));
    } else {
      rk[slot(q)] = key | (first ? kSbFirst : 0u) | (last ? kSbLast : 0u);
      rv[slot(q)] = cval[P0 + jc];
    }
  }
}

struct SbArgs {
  const int4* bdesc;
  const uint32_t* ck;
  const void* cv;
  const uint32_t* rk;
  const void* rv;
  const uint16_t* rp;
  int64_t m;
  const double* u;
  const double* c;  // coef_j = c_j t_j (null: coef_j = t_j)
  double* part;
  int64_t ldp;
  const int32_t* done;
  CgFuse cg;  // inside CG: open the iteration (stop test, beta, d_k)
};

// One DPP step of the segmented scan: (F, S) combined with the pair of the
// source lane that `ctrl` selects (the identity (0, 0) where it selects none).
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_dpp(int& F, double& S) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(S), CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(S), CTRL, ROWS, 0xf, true);
  const int Fp = __builtin_amdgcn_update_dpp(0, F, CTRL, ROWS, 0xf, true);
  const double Sp = __hiloint2double(hi, lo);
  if (!F) S = Sp + S;
  F |= Fp;
}

// Inclusive segmented scan of (start flag f, value s) over the workgroup's
// threads in thread order: S_t = s_t if f_t, else S_{t-1} + s_t.  Within a wave
// by DPP (shifts by 1, 2, 4, 8 inside rows of 16 lanes, then row 15's pair to
// the next row and lane 31's to the upper half), then the waves' totals in wave
// order; the order of additions depends only on the flags, so the result is
// reproducible.
__device__ __forceinline__ double seg_scan(int f, double s, int* wf, double* ws) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int F = f;
  double S = s;
  seg_dpp<0x111, 0xf>(F, S);  // row_shr:1
  seg_dpp<0x112, 0xf>(F, S);  // row_shr:2
  seg_dpp<0x114, 0xf>(F, S);  // row_shr:4
  seg_dpp<0x118, 0xf>(F, S);  // row_shr:8
  seg_dpp<0x142, 0xa>(F, S);  // row_bcast:15 into rows 1 and 3
  seg_dpp<0x143, 0xc>(F, S);  // row_bcast:31 into rows 2 and 3
  if (lane == 63) {
    wf[wid] = F;
    ws[wid] = S;
  }
  __syncthreads();
  // the waves' totals scanned the same way by the first 16 lanes of wave 0;
  // wave w then takes the scan up to wave w - 1
  constexpr int kW = kSbThreads / 64;
  static_assert(kW <= 16, "one DPP row holds the wave totals");
  if (wid == 0) {
    int Fw = lane < kW ? wf[lane] : 1;
    double Sw = lane < kW ? ws[lane] : 0.0;
    seg_dpp<0x111, 0xf>(Fw, Sw);
    seg_dpp<0x112, 0xf>(Fw, Sw);
    seg_dpp<0x114, 0xf>(Fw, Sw);
    seg_dpp<0x118, 0xf>(Fw, Sw);
    if (lane + 1 < kW) ws[kW + lane + 1] = Sw;
  }
  __syncthreads();
  if (!F && wid > 0) S = ws[kW + wid] + S;
  return S;
}

// Sums of a thread's run (its n <= kSbK consecutive non-zeros of one order:
// keys and terms) per segment (column or row: key >> 16; a key's kSbFirst /
// kSbLast flag marks a segment's first / last non-zero).  A segment that starts
// and ends inside the run is stored at out[segment] directly; the run's first
// and last segments may go on in the neighbouring runs and are joined by the
// segmented scan over the threads: the thread holding a segment's last
// non-zero stores the scanned sum of all its pieces (PAD: at out[cpad(segment)]).
// Every thread of the workgroup calls it (barriers inside).
template <bool PAD>
__device__ __forceinline__ void run_sums(const uint32_t (&key)[kSbK], const double (&term)[kSbK],
                                         int n, double* out, double* s_S, int* wf, double* ws) {
  const int tid = threadIdx.x;
  auto at = [](uint32_t kk) {
    const int i = (int)(kk >> 16);
    return PAD ? cpad(i) : i;
  };
  int runs = 0, hi = -1, ti = -1;
  double hs = 0, acc = 0;
  bool first_flag = false, last_flag = false;
#pragma unroll
  for (int k = 0; k < kSbK; ++k) {
    if (k < n) {
      const uint32_t kk = key[k];
      if (k == 0) first_flag = (kk & kSbFirst) != 0;
      if (k == n - 1) last_flag = (kk & kSbLast) != 0;
      if (k == 0 || (kk & kSbFirst)) {  // a new segment starts here
        if (runs == 1) {
          hs = acc;
        } else if (runs > 1) {
          out[ti] = acc;  // started and ended inside this run
        }
        if (runs == 0) hi = at(kk);
        ti = at(kk);
        acc = term[k];
        ++runs;
      } else {
        acc += term[k];
      }
    }
  }
  const bool cont_in = runs > 0 && !first_flag;   // the first segment began earlier
  const bool cont_out = runs > 0 && !last_flag;   // the last one goes on later
  const bool single = runs == 1;
  const double S = seg_scan((single && cont_in) ? 0 : 1, runs > 0 ? acc : 0.0, wf, ws);
  s_S[tid] = S;
  __syncthreads();
  if (runs > 1) out[hi] = cont_in ? s_S[tid - 1] + hs : hs;
  if (runs > 0 && !cont_out) out[ti] = S;
  __syncthreads();
}

template <typename TV>
__global__ __launch_bounds__(kSbThreads) void k_sb_normal(SbArgs a) {
  extern __shared__ double dyn[];  // u (m rows), then the block's partial q (m rows)
  __shared__ double coef[kSbCoefLds];
  __shared__ double sred[2];
  __shared__ double s_S[kSbThreads];
  __shared__ int wf[kSbThreads / 64];
  __shared__ double ws[2 * (kSbThreads / 64)];  // wave totals, then their scan
  // FP32 values: the column-order entries by block-local slot, read back in
  // row order through the references
  constexpr bool kRefs = sb_refs<TV>();
  __shared__ uint32_t skey[kRefs ? kSbEntries : 1];
  __shared__ TV sval[kRefs ? kSbEntries : 1];
  const int64_t m = a.m;
  double* us = dyn;
  double* qs = dyn + ((m + 1) & ~1ll);
  const int tid = threadIdx.x, lane = tid & 63;
  const bool cg_open = a.cg.on && a.cg.k > 0;
  // Requested at once: the done flag, the block's extent, the staged m-vector
  // entries and the CG partial sums.  The block's keys and values (the bulk of
  // the bytes) only once the done flag is known to be clear, so that passes
  // queued after the CG stopped stay cheap.
  const int32_t done0 = a.done ? *a.done : 0;
  const int4 bd = a.bdesc[blockIdx.x];  // first column, columns, non-zeros, first slot
  const int64_t c0 = bd.x, O = bd.w;
  const int ncol = bd.y;
  constexpr int kSt = kSbRows / kSbThreads;
  double st0[kSt], st1[kSt];
#pragma unroll
  for (int q = 0; q < kSt; ++q) {
    const int64_t i = tid + kSbThreads * q;
    const int64_t ic = i < m ? i : 0;
    if (cg_open) {
      st0[q] = a.cg.z[ic];
      st1[q] = a.cg.d_old[ic];
    } else {
      st0[q] = a.u[ic];
    }
  }
  double pre0[4] = {0, 0, 0, 0}, pre1[4] = {0, 0, 0, 0};
  if (cg_open && tid < 64) {
    const int pn = a.cg.np;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = lane + 64 * q;
      const int pc = p < pn ? p : pn - 1;
      pre0[q] = a.cg.prz[2 * (int64_t)pc];
      pre1[q] = a.cg.prz[2 * (int64_t)pc + 1];
    }
  }
  // the scalars of the opening test, written by earlier launches
  double pf_tol2 = 0, pf_rzh = 0;
  int pf_resid = 0, pf_max = 0;
  if (cg_open) {
    pf_tol2 = a.cg.sc[S_CG_TOL2];
    pf_rzh = a.cg.sc[S_CG_RZH0 + (int)((a.cg.k - 1) & 1)];
    pf_resid = a.cg.is[I_CG_RESID];
    pf_max = a.cg.is[I_CG_MAX];
  }
  if (done0) return;
  const int N = bd.z;
  const int K = sb_k(N);
  const int n_mine = tid * K < N ? (N - tid * K < K ? N - tid * K : K) : 0;
  const TV* __restrict__ cvp = (const TV*)a.cv;
  const TV* __restrict__ rvp = (const TV*)a.rv;
  uint32_t ckt[kSbK], rkt[kSbK];
  TV cvt[kSbK], rvt[kSbK];
  uint16_t rpt[kSbK];
#pragma unroll
  for (int k = 0; k < kSbK; ++k) {
    ckt[k] = 0;
    rkt[k] = 0;
    cvt[k] = 0;
    rvt[k] = 0;
    rpt[k] = 0;
    if (k < n_mine) {
      const int64_t p = O + (int64_t)k * kSbThreads + tid;
      ckt[k] = a.ck[p];
      cvt[k] = cvp[p];
      if constexpr (kRefs) {
        rpt[k] = a.rp[p];
      } else {
        rkt[k] = a.rk[p];
        rvt[k] = rvp[p];
      }
    }
  }
  constexpr int kCp = kSbCols / kSbThreads;
  double spre[kCp];
#pragma unroll
  for (int q = 0; q < kCp; ++q) {
    const int lc = tid + kSbThreads * q;
    spre[q] = a.c && lc < ncol ? a.c[c0 + lc] : 1.0;
  }
  if (cg_open) {
    if (tid < 64) {
      const int pn = a.cg.np;
      double s0 = 0, s1 = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool in = lane + 64 * q < pn;
        s0 += in ? pre0[q] : 0.0;
        s1 += in ? pre1[q] : 0.0;
      }
      for (int p = lane + 64 * 4; p < pn; p += 64) {
        s0 += a.cg.prz[2 * p];
        s1 += a.cg.prz[2 * p + 1];
      }
      s0 = lane_group_sum<64>(s0);
      s1 = lane_group_sum<64>(s1);
      if (lane == 0) {
        sred[0] = s0;
        sred[1] = s1;
      }
    }
    __syncthreads();
    const int64_t k = a.cg.k;
    double* sc = a.cg.sc;
    int32_t* is = a.cg.is;
    const double rz = sred[0], rr = sred[1];
    const double crit = pf_resid ? rr : rz;
    const bool stop = k >= pf_max || crit <= pf_tol2 || !(rz > 0);
    const double beta = a.cg.inner == SKIPM_INNER_CG ? rz / pf_rzh : 0.0;
    __syncthreads();
    if (blockIdx.x == 0 && tid == 0) {
      sc[S_CG_RZ] = rz;
      sc[S_V_RR] = rr;
      sc[S_CG_RZH0 + (int)(k & 1)] = rz;
      is[I_CG_ITERS] = (int32_t)k;
      if (stop) is[I_CG_DONE] = 1;
    }
    if (stop) return;
#pragma unroll
    for (int q = 0; q < kSt; ++q) {
      const int64_t i = tid + kSbThreads * q;
      if (i < m) {
        const double di = st0[q] + beta * st1[q];
        us[i] = di;
        if (blockIdx.x == 0) a.cg.d_new[i] = di;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < kSt; ++q) {
      const int64_t i = tid + kSbThreads * q;
      if (i < m) us[i] = st0[q];
    }
  }
  for (int64_t i = tid; i < m; i += kSbThreads) qs[i] = 0.0;
#pragma unroll
  for (int q = 0; q < kCp; ++q) {
    const int lc = tid + kSbThreads * q;
    if (lc < ncol) coef[cpad(lc)] = 0.0;  // columns with no non-zero keep t_j = 0
  }
  if constexpr (kRefs) {
#pragma unroll
    for (int k = 0; k < kSbK; ++k)
      if (k < n_mine) {
        skey[k * kSbThreads + tid] = ckt[k];
        sval[k * kSbThreads + tid] = cvt[k];
      }
  }
  __syncthreads();

  // column phase: t_j
  {
    double term[kSbK];
#pragma unroll
    for (int k = 0; k < kSbK; ++k) term[k] = (double)cvt[k] * us[ckt[k] & kSbLow];
    run_sums<true>(ckt, term, n_mine, coef, s_S, wf, ws);
  }
  if (a.c) {  // coef_j = c_j t_j
#pragma unroll
    for (int q = 0; q < kCp; ++q) {
      const int lc = tid + kSbThreads * q;
      if (lc < ncol) coef[cpad(lc)] = spre[q] * coef[cpad(lc)];
    }
    __syncthreads();
  }
  // row phase: q_i
  {
    double term[kSbK];
    if constexpr (kRefs) {
#pragma unroll
      for (int k = 0; k < kSbK; ++k) {
        term[k] = 0.0;
        if (k < n_mine) {
          const int e = rpt[k] & kRpSlot;
          const uint32_t key = skey[e];  // local column << 16 | row
          rkt[k] = ((key & kSbLow) << 16) | ((rpt[k] & kRpFirst) ? kSbFirst : 0u) |
                   ((rpt[k] & kRpLast) ? kSbLast : 0u);
          term[k] = (double)sval[e] * coef[cpad((int)(key >> 16))];
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < kSbK; ++k)
        term[k] = (double)rvt[k] * coef[cpad((int)(rkt[k] & kSbLow))];
    }
    run_sums<false>(rkt, term, n_mine, qs, s_S, wf, ws);
  }
  double* out = a.part + (int64_t)blockIdx.x * a.ldp;
  for (int64_t i = tid; i < m; i += kSbThreads) out[i] = qs[i];
}

}  // namespace

int64_t sb_max_blocks(int64_t n, int64_t nnz) {
  return (n + kSbCols - 1) / kSbCols + nnz / kSbCap + 1;
}

int64_t sb_max_slots(int64_t n, int64_t nnz) {
  return nnz + sb_max_blocks(n, nnz) * (int64_t)(kSbThreads - 1);
}

// Greedy cut on the host: a column joins the current block unless the block
// already has kSbCols columns or would pass kSbEntries non-zeros with it (a
// column has at most m <= kMaxM < kSbEntries).  Every block but the last has
// kSbCols columns or more than kSbCap non-zeros, hence sb_max_blocks.  Block
// b's region of the keyed copies holds K_b * 1024 slots, K_b = ceil(N_b /
// 1024) (fewer than N_b + 1024), hence sb_max_slots.  bdesc[b] = (first
// column, columns, non-zeros, first slot); returns the number of slots.
int64_t sb_partition(const SparseA& A, std::vector<int32_t>* bdesc, hipStream_t st) {
  const int64_t n = A.n;
  std::vector<int32_t> cp((size_t)n + 1);
  if (hipMemcpyAsync(cp.data(), A.colptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return -1;
  std::vector<int64_t> bcol{0};
  int64_t start = 0;
  for (int64_t c = 0; c < n; ++c) {
    if (c - start == kSbCols || (int64_t)cp[c + 1] - cp[start] > kSbEntries) {
      bcol.push_back(c);
      start = c;
    }
  }
  bcol.push_back(n);
  const size_t nbk = bcol.size() - 1;
  bdesc->assign(4 * nbk, 0);
  int64_t off = 0;
  for (size_t b = 0; b < nbk; ++b) {
    const int64_t N = (int64_t)cp[bcol[b + 1]] - cp[bcol[b]];
    (*bdesc)[4 * b] = (int32_t)bcol[b];
    (*bdesc)[4 * b + 1] = (int32_t)(bcol[b + 1] - bcol[b]);
    (*bdesc)[4 * b + 2] = (int32_t)N;
    (*bdesc)[4 * b + 3] = (int32_t)off;
    off += (int64_t)sb_k(N) * kSbThreads;
  }
  return off;
}

void sb_fill(SparseA* A, const int32_t* bdesc, uint32_t* ck, void* cv, uint32_t* rk, void* rv,
             uint16_t* rp, int32_t* bad, hipStream_t st) {
  const int4* bd = (const int4*)bdesc;
  if (A->vdt == SKIPM_F64)
    hipLaunchKernelGGL(k_sb_sort<double>, dim3((unsigned)A->nbk), dim3(1024), 0, st, A->colptr,
                       A->rowidx, (const double*)A->cval, bd, ck, (double*)cv, rk, (double*)rv,
                       rp, bad);
  else
    hipLaunchKernelGGL(k_sb_sort<float>, dim3((unsigned)A->nbk), dim3(1024), 0, st, A->colptr,
                       A->rowidx, (const float*)A->cval, bd, ck, (float*)cv, rk, (float*)rv, rp,
                       bad);
  A->bdesc = bdesc;
  A->ck = ck;
  A->cv = cv;
  A->rk = rk;
  A->rv = rv;
  A->rp = rp;
}

int launch_sb_normal(const SparseA& A, const double* u, const double* c, double* part,
                     int64_t ldp, const int32_t* done, hipStream_t st, const CgFuse* cg) {
  if (A.m > kMaxM || A.nbk < 1 || ldp < A.m) return -1;
  SbArgs a{};
  if (cg) a.cg = *cg;
  a.bdesc = (const int4*)A.bdesc;
  a.ck = A.ck;
  a.cv = A.cv;
  a.rk = A.rk;
  a.rv = A.rv;
  a.rp = A.rp;
  a.m = A.m;
  a.u = u;
  a.c = c;
  a.part = part;
  a.ldp = ldp;
  a.done = done;
  const size_t lds = (size_t)2 * ((A.m + 1) & ~1ll) * sizeof(double);
  if (A.vdt == SKIPM_F64)
    hipLaunchKernelGGL(k_sb_normal<double>, dim3((unsigned)A.nbk), dim3(kSbThreads), lds, st, a);
  else
    hipLaunchKernelGGL(k_sb_normal<float>, dim3((unsigned)A.nbk), dim3(kSbThreads), lds, st, a);
  return 0;
}

}  // namespace skipm
