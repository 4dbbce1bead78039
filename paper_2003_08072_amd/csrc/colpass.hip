// One streaming pass over a dense column-major matrix (A, the sketch B, or the
// inverse Gram matrix), doing per column j:
//     t_j = a_j^T u                      (a dot product down the column)
//     acc += coef_j(t_j, ...) * a_j      (an axpy of the same column)
// so that a product like A D^2 A^T u needs exactly one read of A.  Modes:
//   COL_NORMAL    coef_j = d2_j t_j                  -> A D^2 A^T u  (CG product)
//   COL_PROLOGUE  t_j = a_j^T y,  r_d,j = t_j + s_j - c_j,  d2_j = x_j / s_j,
//                 acc1 += x_j a_j,  acc2 += (sigma mu / s_j + d2_j r_d,j) a_j
//                 -> A x and A (sigma mu S^{-1} 1 + D^2 r_d); with them
//                    r_p = A x - b and p = b - A(sigma mu / s + d2 r_d), which is
//                    eq. pdef with its A x terms cancelled.
//   COL_EPILOGUE  t_j = a_j^T dy, ds_j = -r_d,j - t_j (eq. delshat),
//                 acc += d2_j t_j a_j  -> A D^2 A^T dy (for g = A D^2 A^T dy - p)
//   COL_DOT       t_j only (a GEMV with the transpose)
//   COL_AXPY      no dot: acc += coef_j a_j with coef given   -> A coef  (a GEMV)
//
// Layout: a group of G lanes owns one column at a time; lane l of the group
// holds rows (r*G + l)*V .. +V-1 for r < R, read as one 16-byte vector per r,
// so a group reads a column with fully coalesced 16-byte-per-lane loads.  The
// column's dot is summed over the G lanes by DPP moves.  Each workgroup streams a
// contiguous range of columns (next column prefetched into registers), keeps
// its accumulators in registers, folds its waves together through LDS in a
// fixed order and writes one partial vector; launch_finish sums the partials
// of all workgroups in a fixed order, so results are bitwise reproducible.
#include <hip/hip_ext.h>
#include <string.h>

#include <utility>

#include "common.h"

namespace skipm {

namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

template <typename TA>
struct Vec;
template <>
struct Vec<double> {
  static constexpr int V = 2;
  typedef dvec2 type;
};
template <>
struct Vec<float> {
  static constexpr int V = 4;
  typedef fvec4 type;
};
// bfloat16 values as raw 16-bit patterns (the upper half of an FP32 word)
struct bf16_t {
  unsigned short bits;
};
typedef unsigned short hvec8 __attribute__((ext_vector_type(8)));
template <>
struct Vec<bf16_t> {
  static constexpr int V = 8;
  typedef hvec8 type;
};

// one element of a loaded vector, widened exactly to FP64
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(unsigned short b) {
  return (double)__uint_as_float((unsigned)b << 16);
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
  return lane_group_sum<G>(v);
}

struct Args {
  const void* A;
  int64_t lda, m, n, cpb;
  const void* u;
  const double* x;
  const double* s;
  const double* c;
  const double* rd;
  const void* d2;
  double* rd_out;
  double* d2_out;
  float* d2f_out;
  double* ds_out;
  void* t_out;
  void* part;
  int64_t ldp;
  double* red;
  const double* sc;
  const int32_t* done;
  CgFuse cg;
  int shape = 0;  // grouped launches: the matrix's lane-group shape (index into kGShapes)
};

// LDS of one pass: the wave fold's buffer (with many waves, each wave parks
// its sums in its own LDS row and the rows are added in one step; otherwise,
// or when that would take more than 64 KB, the waves add into one row in
// turn), per-wave scalar sums and the CG's two opening sums.
template <typename TA, typename TC, int G, int R, int MODE, int NT>
struct ColLds {
  static constexpr int V = Vec<TA>::V;
  static constexpr int NW = NT / 64;
  static constexpr int NACC = MODE == COL_PROLOGUE ? 2 : (MODE == COL_DOT ? 0 : 1);
  static constexpr int NACC1 = NACC > 0 ? NACC : 1;
  static constexpr int LROWS = G * R * V;
  static constexpr bool kOneStep = NW >= 8 && NW * LROWS * sizeof(TC) <= 65536;
  static constexpr int kLbuf = kOneStep ? NW * LROWS : NACC1 * LROWS;  // TC entries
  static constexpr size_t kSred = (size_t)kLbuf * sizeof(TC);          // byte offsets
  static constexpr size_t kCgs = kSred + (size_t)NW * 4 * sizeof(double);
  static constexpr size_t kBytes = kCgs + 2 * sizeof(double);
};

// The pass of workgroup `bid` of one matrix (its column range, its partial):
// the body of k_colpass, and of the grouped kernels for each matrix of a
// group; `smem` is the caller's LDS of at least ColLds<...>::kBytes.
template <typename TA, typename TC, int G, int R, int MODE, int NT, bool STREAM>
__device__ __forceinline__ void colpass_body(const Args& a, const int bid, char* smem) {
  typedef ColLds<TA, TC, G, R, MODE, NT> L;
  constexpr int V = Vec<TA>::V;
  typedef typename Vec<TA>::type VT;
  constexpr int NGW = 64 / G;
  constexpr int NW = NT / 64;
  constexpr int NACC = L::NACC;
  constexpr int NACC1 = L::NACC1;
  constexpr int LROWS = L::LROWS;
  constexpr bool kOneStep = L::kOneStep;
  TC* lbuf = (TC*)smem;
  double(*sred)[4] = (double(*)[4])(smem + L::kSred);

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = lane / G, lg = lane % G;
  const int slot = wid * NGW + grp;
  constexpr int NSLOT = NW * NGW;
  const int64_t c0 = (int64_t)bid * a.cpb;
  const int64_t c1 = c0 + a.cpb < a.n ? c0 + a.cpb : a.n;
  const TA* __restrict__ A = (const TA*)a.A;
  const TC* __restrict__ u = (const TC*)a.u;
  const TC* __restrict__ d2 = (const TC*)a.d2;

  bool valid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) valid[r] = (int64_t)(r * G + lg) * V < a.lda;
  // STREAM (a pass over an A larger than the Infinity Cache): non-temporal
  // loads, which stream from HBM faster than cached ones and leave the caches
  // to what the small CG kernels reuse every iteration.  A matrix that fits
  // the cache is read with ordinary loads and stays resident.
  auto load_col = [&](VT* dst, const int64_t col) {
    const VT* p = (const VT*)(A + col * a.lda);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (valid[r]) dst[r] = STREAM ? __builtin_nontemporal_load(&p[r * G + lg]) : p[r * G + lg];
  };
  // The first columns are requested before anything else: they depend on
  // nothing, so their latency overlaps the set-up below.  Two columns per trip
  // later, the next two prefetched while these are used (up to four columns
  // per lane group in flight).
  // PD columns per trip (2 * PD per lane group in flight).  Four per trip for
  // BF16 columns (one 16-byte load per lane each) measured no faster than two.
  constexpr int PD = 2;
  VT cv[PD][R], nv[PD][R];
#pragma unroll
  for (int q = 0; q < PD; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cv[q][r] = (VT)0;
      nv[q][r] = (VT)0;
    }
  int64_t col = c0 + slot;
#pragma unroll
  for (int q = 0; q < PD; ++q)
    if (col + q * NSLOT < c1) load_col(cv[q], col + q * NSLOT);

  const bool cg = a.cg.on != 0;
  const bool cg_dir = cg && MODE == COL_NORMAL && a.cg.k > 0;
  // CG close pass: d, r, q, z, x at the slot's first column are requested
  // with the column itself (a slot of that pass owns at most one column; a
  // later one loads its own)
  const int64_t col_first = col;
  double pf_d = 0, pf_r = 0, pf_q = 0, pf_z = 0, pf_x = 0;
  if (MODE == COL_DOT && cg) {
    const int64_t jc = col < a.n ? col : a.n - 1;
    pf_d = a.cg.d[jc];
    pf_r = a.cg.r[jc];
    pf_q = a.cg.q[jc];
    pf_z = a.cg.zz[jc];
    pf_x = a.cg.x[jc];
  }
  TC uu[R][V];
  double dold[R][V];
  TC acc1[R][V], acc2[R][V];
  // u, and z_k and d_{k-1} when the pass opens a CG iteration (d_k is formed
  // once beta_k is known).  Every load is in bounds (rows past lda read row
  // 0; their values are never used) and no select waits on a loaded value
  // before the done check below.
  double zraw[R][V];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row0 = (int64_t)(r * G + lg) * V;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int64_t idx = valid[r] ? row0 + e : 0;
      uu[r][e] = MODE != COL_AXPY ? u[idx] : (TC)0;
      acc1[r][e] = 0;
      acc2[r][e] = 0;
    }
  }
  if (cg_dir) {  // z and d are read (and defined) only when a CG iteration opens
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row0 = (int64_t)(r * G + lg) * V;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int64_t idx = valid[r] ? row0 + e : 0;
        zraw[r][e] = a.cg.z[idx];
        dold[r][e] = a.cg.d_old[idx];
      }
    }
  }
  // the partial sums the pass opens with (r^T z, r^T r of the last iteration,
  // or d^T q of this one), requested by wave 0 with the first columns: up to
  // kPre per lane here, any further ones in a loop below
  constexpr int kPre = 8;
  const bool cg_open = cg && MODE == COL_NORMAL && a.cg.k > 0;
  const bool cg_close = cg && MODE == COL_DOT;
  const double* pv = cg_open ? a.cg.prz : (cg_close ? a.cg.pdq : nullptr);
  const int pn = cg_open ? a.cg.np : (cg_close ? a.cg.nf : 0);
  const int pst = cg_open ? 2 : 1;
  double pre0[kPre], pre1[kPre];
#pragma unroll
  for (int q = 0; q < kPre; ++q) {
    pre0[q] = 0.0;
    pre1[q] = 0.0;
  }
  if (wid == 0 && pn > 0) {
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int p = lane + 64 * q;
      const int pc = p < pn ? p : pn - 1;
      pre0[q] = pv[(int64_t)pc * pst];
      pre1[q] = pv[(int64_t)pc * pst + (cg_open ? 1 : 0)];  // unused unless cg_open
    }
  }
  // the scalars the opening test (or the closing step) reads, requested with
  // the partials: the stopping threshold, the cap and r^T z of the previous
  // iteration (of this one when closing), all written by earlier launches
  double pf_tol2 = 0, pf_rzh = 0;
  int pf_resid = 0, pf_max = 0;
  if (cg_open) {
    pf_tol2 = a.cg.sc[S_CG_TOL2];
    pf_rzh = a.cg.sc[S_CG_RZH0 + (int)((a.cg.k - 1) & 1)];
    pf_resid = a.cg.is[I_CG_RESID];
    pf_max = a.cg.is[I_CG_MAX];
  } else if (cg_close) {
    pf_rzh = a.cg.sc[S_CG_RZH0 + (int)(a.cg.k & 1)];
  }
  // the done flag of a finished CG is read only now, so that its latency
  // overlaps that of the loads above (all in bounds)
  if (a.done && *a.done) return;
  // an empty asm "redefines" the prefetched partials here, so that their sums
  // below stay below the done check (the compiler would otherwise start them
  // early, and the wait for those loads would come before the flag's load)
#pragma unroll
  for (int q = 0; q < kPre; ++q) asm volatile("" : "+v"(pre0[q]), "+v"(pre1[q]));
  asm volatile("" : "+v"(pf_tol2), "+v"(pf_rzh), "+v"(pf_resid), "+v"(pf_max));
  if (cg_dir) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int e = 0; e < V; ++e) uu[r][e] = (TC)zraw[r][e];
  }

  // fused CG bookkeeping at the start of the pass (every block computes the
  // same sums in the same order, so every block takes the same decision)
  double* cgs = (double*)(smem + L::kCgs);
  double cg_beta = 0, cg_alpha = 0;
  if (cg && (MODE == COL_NORMAL || MODE == COL_DOT)) {
    const int64_t k = a.cg.k;
    if (wid == 0) {
      // sum over p = lane, lane + 64, ... in that order, then over the wave
      double s0 = 0, s1 = 0;
#pragma unroll
      for (int q = 0; q < kPre; ++q) {
        const bool in = lane + 64 * q < pn;
        s0 += in ? pre0[q] : 0.0;
        s1 += in && cg_open ? pre1[q] : 0.0;
      }
      for (int p = lane + 64 * kPre; p < pn; p += 64) {
        s0 += pv[(int64_t)p * pst];
        if (cg_open) s1 += pv[(int64_t)p * pst + 1];
      }
      s0 = lane_group_sum<64>(s0);
      s1 = lane_group_sum<64>(s1);
      if (lane == 0) {
        cgs[0] = s0;
        cgs[1] = s1;
      }
    }
    __syncthreads();
    double* sc = a.cg.sc;
    int32_t* is = a.cg.is;
    if (MODE == COL_NORMAL && k > 0) {
      const double rz = cgs[0], rr = cgs[1];
      const double crit = pf_resid ? rr : rz;
      const bool stop = k >= pf_max || crit <= pf_tol2 || !(rz > 0);
      cg_beta = a.cg.inner == SKIPM_INNER_CG ? rz / pf_rzh : 0.0;
      if (bid == 0 && threadIdx.x == 0) {
        sc[S_CG_RZ] = rz;
        sc[S_V_RR] = rr;
        sc[S_CG_RZH0 + (int)(k & 1)] = rz;
        is[I_CG_ITERS] = (int32_t)k;
        if (stop) is[I_CG_DONE] = 1;
      }
      if (stop) return;
    } else if (MODE == COL_DOT) {
      const double dq = cgs[0];
      if (!(dq > 0)) {  // breakdown: the operator lost positive definiteness numerically
        if (bid == 0 && threadIdx.x == 0) is[I_CG_DONE] = 1;
        return;
      }
      cg_alpha = a.cg.inner == SKIPM_INNER_RICHARDSON ? 1.0 : pf_rzh / dq;
    }
  }
  double cg_pz = 0, cg_pr = 0;
  if (cg_dir) {  // d_k = z_k + beta_k d_{k-1}; block 0 stores it
    const bool store = bid == 0 && wid == 0 && grp == 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row0 = (int64_t)(r * G + lg) * V;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double dk = (double)uu[r][e] + cg_beta * dold[r][e];
        if (store && valid[r]) a.cg.d_new[row0 + e] = dk;
        uu[r][e] = (TC)dk;
      }
    }
  }
  double mu = 0, sigma = 0;
  if (MODE == COL_PROLOGUE) {
    mu = a.sc[S_MU];
    sigma = a.sc[S_SIGMA];
  }
  double sr0 = 0, sr1 = 0, sr2 = 0;

  // Per-column work on the R vectors of column `col` held by this lane.
  auto process = [&](const VT* cur, const int64_t col) {
      TC dot = 0;
      if (MODE != COL_AXPY) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!valid[r]) continue;
#pragma unroll
          for (int e = 0; e < V; ++e) dot += (TC)widen(cur[r][e]) * uu[r][e];
        }
        dot = group_sum<G>(dot);
      }
      if (MODE == COL_AXPY) {
        const TC coef = d2[col];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) acc1[r][e] += coef * (TC)widen(cur[r][e]);
      } else if (MODE == COL_DOT) {
        if (cg) {
          if (lg == 0) {  // w_j = (Q^{-1} q)_j: update x, r, z at j
            const bool pf = col == col_first;
            const double dj = pf ? pf_d : a.cg.d[col];
            const double rj = (pf ? pf_r : a.cg.r[col]) - cg_alpha * (pf ? pf_q : a.cg.q[col]);
            const double zj = (pf ? pf_z : a.cg.zz[col]) - cg_alpha * (double)dot;
            a.cg.x[col] = (pf ? pf_x : a.cg.x[col]) + cg_alpha * dj;
            a.cg.r[col] = rj;
            a.cg.zz[col] = zj;
            cg_pz += rj * zj;
            cg_pr += rj * rj;
          }
        } else if (lg == 0) {
          ((TC*)a.t_out)[col] = dot;
        }
      } else if (MODE == COL_NORMAL) {
        const TC coef = d2 ? d2[col] * dot : dot;
        if (a.t_out && lg == 0) ((TC*)a.t_out)[col] = dot;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) acc1[r][e] += coef * (TC)widen(cur[r][e]);
      } else if (MODE == COL_EPILOGUE) {
        const double t = (double)dot;
        const double dsj = -a.rd[col] - t;
        const double coef = ((const double*)a.d2)[col] * t;
        if (lg == 0) a.ds_out[col] = dsj;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) acc1[r][e] += (TC)(coef * widen(cur[r][e]));
      } else {  // COL_PROLOGUE
        const double t = (double)dot;
        const double xj = a.x[col], sj = a.s[col], cj = a.c[col];
        const double rdj = t + sj - cj;
        const double d2j = xj / sj;
        const double ej = sigma * mu / sj + d2j * rdj;
        if (lg == 0) {
          a.rd_out[col] = rdj;
          a.d2_out[col] = d2j;
          if (a.d2f_out) a.d2f_out[col] = (float)d2j;
          sr0 += rdj * rdj;
          sr1 += cj * xj;
          sr2 += xj * sj;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) {
            acc1[r][e] += (TC)(xj * widen(cur[r][e]));
            acc2[r][e] += (TC)(ej * widen(cur[r][e]));
          }
      }
  };
  while (col < c1) {
#pragma unroll
    for (int q = 0; q < PD; ++q)
      if (col + (PD + q) * NSLOT < c1) load_col(nv[q], col + (PD + q) * NSLOT);
    process(cv[0], col);
#pragma unroll
    for (int q = 1; q < PD; ++q)
      if (col + q * NSLOT < c1) process(cv[q], col + q * NSLOT);
#pragma unroll
    for (int q = 0; q < PD; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) cv[q][r] = nv[q][r];
    col += PD * NSLOT;
  }

  if (MODE == COL_PROLOGUE) {
    // workgroup sums of the per-column scalars (only lg == 0 lanes are non-zero)
    sr0 = group_sum<64>(sr0);
    sr1 = group_sum<64>(sr1);
    sr2 = group_sum<64>(sr2);
    if (lane == 0) {
      sred[wid][0] = sr0;
      sred[wid][1] = sr1;
      sred[wid][2] = sr2;
    }
  }
  if (NACC == 0) {
    if (cg && MODE == COL_DOT) {  // block partials of r^T z, r^T r in a fixed order
      cg_pz = lane_group_sum<64>(cg_pz);
      cg_pr = lane_group_sum<64>(cg_pr);
      if (lane == 0) {
        sred[wid][0] = cg_pz;
        sred[wid][1] = cg_pr;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double t0 = 0, t1 = 0;
        for (int w = 0; w < NW; ++w) {
          t0 += sred[w][0];
          t1 += sred[w][1];
        }
        a.cg.prz_out[2 * bid] = t0;
        a.cg.prz_out[2 * bid + 1] = t1;
      }
    }
    return;
  }
  // fold the groups of a wave (same rows) together
#pragma unroll
  for (int off = G; off < 64; off <<= 1) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        acc1[r][e] += __shfl_xor(acc1[r][e], off, 64);
        if (NACC > 1) acc2[r][e] += __shfl_xor(acc2[r][e], off, 64);
      }
  }
  TC* part = (TC*)a.part + (int64_t)bid * NACC * a.ldp;
  if constexpr (kOneStep) {
    // each row of the partial is the sum over waves in wave order: the same
    // order, hence the same rounding, as the turn-by-turn fold below
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
      if (grp == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e)
            lbuf[wid * LROWS + (r * G + lg) * V + e] = k == 0 ? acc1[r][e] : acc2[r][e];
      }
      __syncthreads();
      for (int64_t i = threadIdx.x; i < a.m; i += NT) {
        TC sum = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += lbuf[w * LROWS + i];
        part[k * a.ldp + i] = sum;
      }
      if (k + 1 < NACC) __syncthreads();
    }
  } else {
    for (int w = 0; w < NW; ++w) {
      if (wid == w && grp == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const int idx = (r * G + lg) * V + e;
            lbuf[idx] = (w == 0 ? (TC)0 : lbuf[idx]) + acc1[r][e];
            if (NACC > 1)
              lbuf[(NACC1 - 1) * LROWS + idx] =
                  (w == 0 ? (TC)0 : lbuf[(NACC1 - 1) * LROWS + idx]) + acc2[r][e];
          }
      }
      __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < a.m; i += NT) {
      part[i] = lbuf[i];
      if (NACC > 1) part[a.ldp + i] = lbuf[(NACC1 - 1) * LROWS + i];
    }
  }
  if (MODE == COL_PROLOGUE && threadIdx.x == 0) {
    double t0 = 0, t1 = 0, t2 = 0;
    for (int w = 0; w < NW; ++w) {
      t0 += sred[w][0];
      t1 += sred[w][1];
      t2 += sred[w][2];
    }
    a.red[bid * 8 + 0] = t0;
    a.red[bid * 8 + 1] = t1;
    a.red[bid * 8 + 2] = t2;
  }
}

template <typename TA, typename TC, int G, int R, int MODE, int NT, bool STREAM>
__global__ __launch_bounds__(NT) void k_colpass(Args a) {
  __shared__ __attribute__((aligned(16))) char smem[ColLds<TA, TC, G, R, MODE, NT>::kBytes];
  colpass_body<TA, TC, G, R, MODE, NT, STREAM>(a, blockIdx.x, smem);
}

// B[:, b] = sum over the (sorted) items of bucket b of sign * d_j * A[:, j]
// (d_j = dsc_j, or sqrt(dsc_j) when dsc holds d^2)
template <typename TA, int G, int R, int NT>
__global__ __launch_bounds__(NT) void k_sketch(const TA* __restrict__ A, int64_t lda, int s,
                                               const double* __restrict__ dsc, int is_d2,
                                               const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ perm,
                                               const int8_t* __restrict__ sign, int w,
                                               double* __restrict__ B, int64_t ldb) {
  constexpr int V = Vec<TA>::V;
  typedef typename Vec<TA>::type VT;
  constexpr int NGW = 64 / G;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = lane / G, lg = lane % G;
  const int gslot = (blockIdx.x * (NT / 64) + wid) * NGW + grp;
  const int nslot = gridDim.x * (NT / 64) * NGW;
  bool valid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) valid[r] = (int64_t)(r * G + lg) * V < lda;
  for (int b = gslot; b < w; b += nslot) {
    double acc[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int e = 0; e < V; ++e) acc[r][e] = 0;
    // The items' metadata (column, coefficient) is fetched G items at a time,
    // one per lane of the group, and handed round with shuffles; only the
    // column loads are left on the chain, one column requested ahead.  The
    // columns are added in item order.
    const int beg = ptr[b], end = ptr[b + 1];
    VT cur[R], nxt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cur[r] = (VT)0;
      nxt[r] = (VT)0;
    }
    for (int it0 = beg; it0 < end; it0 += G) {
      const int itl = it0 + lg;
      long long jl = 0;
      double coefl = 0.0;
      if (itl < end) {
        const int item = perm[itl];
        jl = item / s;
        const double dj = dsc[jl];
        coefl = (double)sign[item] * (is_d2 ? sqrt(dj) : dj);
      }
      const int cnt = end - it0 < G ? end - it0 : G;
      {
        const long long j0 = __shfl(jl, 0, G);
        const VT* p = (const VT*)(A + j0 * lda);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (valid[r]) cur[r] = p[r * G + lg];
      }
      for (int q = 0; q < cnt; ++q) {
        const double coef = __shfl(coefl, q, G);
        if (q + 1 < cnt) {
          const long long jn = __shfl(jl, q + 1, G);
          const VT* p = (const VT*)(A + jn * lda);
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (valid[r]) nxt[r] = p[r * G + lg];
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (valid[r])
#pragma unroll
            for (int e = 0; e < V; ++e) acc[r][e] += coef * widen(cur[r][e]);
#pragma unroll
        for (int r = 0; r < R; ++r) cur[r] = nxt[r];
      }
    }
    double* out = B + (int64_t)b * ldb;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (valid[r]) {
        const int64_t row0 = (int64_t)(r * G + lg) * V;
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (row0 + e < ldb) out[row0 + e] = acc[r][e];
      }
  }
}

// Partials are summed over the block axis by 16 block-lanes x 16 rows per
// workgroup, then the 16 block-lane sums are added in a fixed tree order.
template <typename TP>
__device__ __forceinline__ void finish_body(const TP* __restrict__ part, int64_t ldp,
                                            int64_t off, int nblk, int64_t m, double scale,
                                            const double* __restrict__ add, double beta,
                                            double* __restrict__ out,
                                            const int32_t* __restrict__ done) {
  __shared__ double tile[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + tx;
  // The first 16 partials per thread are requested at once and before the
  // done flag is read: addresses clamped in bounds, no branches around the
  // loads (so they are all in flight together); terms past nblk are scaled
  // by 0.  Added in block order.
  const int64_t ic = i < m ? i : m - 1;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int b = ty + 16 * q < nblk ? ty + 16 * q : nblk - 1;
    v[q] = (double)part[(int64_t)b * ldp + off + ic];
  }
  if (done && *done) return;
  double acc = 0;
  if (i < m) {
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += v[q] * (ty + 16 * q < nblk ? 1.0 : 0.0);
    for (int b = ty + 256; b < nblk; b += 16) acc += (double)part[(int64_t)b * ldp + off + i];
  }
  tile[ty][tx] = acc;
  __syncthreads();
  for (int h = 8; h > 0; h >>= 1) {
    if (ty < h) tile[ty][tx] += tile[ty + h][tx];
    __syncthreads();
  }
  if (ty == 0 && i < m) {
    double v = scale * tile[0][tx];
    if (add) v += beta * add[i];
    out[i] = v;
  }
}

template <typename TP>
__global__ __launch_bounds__(256) void k_finish(const TP* __restrict__ part, int64_t ldp,
                                                int64_t off, int nblk, int64_t m, double scale,
                                                const double* __restrict__ add, double beta,
                                                double* __restrict__ out,
                                                const int32_t* __restrict__ done) {
  finish_body<TP>(part, ldp, off, nblk, m, scale, add, beta, out, done);
}

// Two finishes of the same partials in one launch (blockIdx.y picks the set).
struct FinishSet {
  int64_t off;
  double scale;
  const double* add;
  double beta;
  double* out;
};
__global__ __launch_bounds__(256) void k_finish2(const double* __restrict__ part, int64_t ldp,
                                                 int nblk, int64_t m, FinishSet f0, FinishSet f1) {
  const FinishSet& f = blockIdx.y == 0 ? f0 : f1;
  finish_body<double>(part, ldp, f.off, nblk, m, f.scale, f.add, f.beta, f.out, nullptr);
}

// k_finish for the fused CG: out = sum of the partials, and per workgroup the
// partial sum of dvec_i out_i over its 16 rows, in row order.  Workgroup `bid`
// of one matrix (the body of k_finish_dot and of k_finish_dot_grouped).
__device__ __forceinline__ void finish_dot_body(const double* __restrict__ part, int64_t ldp,
                                                int nblk, int64_t m,
                                                const double* __restrict__ dvec,
                                                double* __restrict__ out,
                                                double* __restrict__ dq_out,
                                                const int32_t* __restrict__ done, const int bid) {
  __shared__ double tile[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i = (int64_t)bid * 16 + tx;
  // as in k_finish: 16 partials per thread in flight before the done flag
  const int64_t ic = i < m ? i : m - 1;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int b = ty + 16 * q < nblk ? ty + 16 * q : nblk - 1;
    v[q] = part[(int64_t)b * ldp + ic];
  }
  if (done && *done) return;
  double acc = 0;
  if (i < m) {
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += v[q] * (ty + 16 * q < nblk ? 1.0 : 0.0);
    for (int b = ty + 256; b < nblk; b += 16) acc += part[(int64_t)b * ldp + i];
  }
  tile[ty][tx] = acc;
  __syncthreads();
  for (int h = 8; h > 0; h >>= 1) {
    if (ty < h) tile[ty][tx] += tile[ty + h][tx];
    __syncthreads();
  }
  if (ty == 0) {
    const double v = tile[0][tx];
    if (i < m) out[i] = v;
    tile[1][tx] = i < m ? dvec[i] * v : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int c = 0; c < 16; ++c) s += tile[1][c];
    dq_out[bid] = s;
  }
}

__global__ __launch_bounds__(256) void k_finish_dot(const double* __restrict__ part, int64_t ldp,
                                                    int nblk, int64_t m,
                                                    const double* __restrict__ dvec,
                                                    double* __restrict__ out,
                                                    double* __restrict__ dq_out,
                                                    const int32_t* __restrict__ done) {
  finish_dot_body(part, ldp, nblk, m, dvec, out, dq_out, done, blockIdx.x);
}

// k_finish_dot over the LPs of a grouped CG; LP i at iteration kstart[i] + j
// takes args[2 i + (k & 1)].
__global__ __launch_bounds__(256) void k_finish_dot_grouped(const FinishDotArgs* __restrict__ args,
                                                            const int32_t* __restrict__ first,
                                                            int nmat,
                                                            const int64_t* __restrict__ kstart,
                                                            int j) {
  int lo = 0, hi = nmat - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const FinishDotArgs& f = args[2 * lo + (int)((kstart[lo] + j) & 1)];
  finish_dot_body(f.part, f.ldp, f.nblk, f.m, f.dvec, f.out, f.dq_out, f.done,
                  (int)blockIdx.x - first[lo]);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
struct Shape {
  int G, R;
};

// g32: the column passes also take lane groups of three vectors per lane, of
// 16 lanes for 32V < lda <= 48V rows and of 32 lanes for 64V < lda <= 96V
// (at most a third or a quarter of the lanes idle, where 64 lanes with one or
// two vectors leave up to half idle: a pass that is bound by the bytes in
// flight per CU gets up to half as many again); the sketch keeps the 16 /
// 64-lane shapes.
Shape pick_shape(int64_t lda, int V, bool g32 = false) {
  if (lda <= 16 * V) return {16, 1};
  if (lda <= 32 * V) return {16, 2};
  if (g32 && lda > 32 * V && lda <= 48 * V) return {16, 3};
  if (g32 && lda > 64 * V && lda <= 96 * V) return {32, 3};
  const int64_t per = 64 * V;
  const int64_t R = (lda + per - 1) / per;
  static const int opts[] = {1, 2, 3, 4, 6, 8, 12, 16};
  for (int o : opts)
    if (o >= R) return {64, o};
  return {0, 0};
}

// Block size from an estimate of the VGPRs a lane needs (u and accumulators in
// the compute type, four 16-byte column buffers, ~32 for addressing, ~32 more
// for the prologue's per-column terms, 8 more when FP32 columns are widened to
// FP64, 24 per row vector when BF16 columns are: eight FP64 values from one
// 16-byte load): 1024 threads need <= 128 VGPRs, 512 threads <= 256.  The estimate
// puts every instantiation that the compiler would have to spill to scratch
// at the smaller block.  DOT passes write no partial sums, so they use small
// blocks and many of them.
constexpr int threads_for(int mode, int R, int V, int tc_bytes, int G = 64) {
  const int nacc = mode == COL_PROLOGUE ? 2 : (mode == COL_DOT ? 0 : 1);
  const int est = (1 + nacc) * R * V * tc_bytes / 4 + 16 * R + 32 +
                  (mode == COL_PROLOGUE ? 32 : 0) + (V == 4 && tc_bytes == 8 ? 8 : 0) +
                  (V == 8 ? 24 * R : 0);
  if (mode == COL_DOT) return 256;
  // 16- and 32-lane groups of three vectors: 768 threads when three waves per
  // SIMD fit (<= 168 VGPRs)
  if (G < 64 && R == 3 && est <= 168) return 768;
  return est <= 128 ? 1024 : (est <= 256 ? 512 : 256);
}

template <typename TA, typename TC, int MODE, int G, int R, bool STREAM>
void launch_one(const Args& a, int nblk, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  constexpr int NT = threads_for(MODE, R, Vec<TA>::V, (int)sizeof(TC), G);
  if (e0)  // events stamped by the runtime with the kernel's own start and end
    hipExtLaunchKernelGGL((k_colpass<TA, TC, G, R, MODE, NT, STREAM>), dim3(nblk), dim3(NT), 0,
                          st, e0, e1, 0, a);
  else
    hipLaunchKernelGGL((k_colpass<TA, TC, G, R, MODE, NT, STREAM>), dim3(nblk), dim3(NT), 0, st,
                       a);
}

// the passes over A that may take non-temporal loads (STREAM)
constexpr bool stream_mode(int mode) {
  return mode == COL_NORMAL || mode == COL_PROLOGUE || mode == COL_EPILOGUE || mode == COL_DOT;
}

template <typename TA, typename TC, int MODE>
int dispatch(const Args& a, int nblk, bool stream, hipStream_t st, hipEvent_t e0 = nullptr,
             hipEvent_t e1 = nullptr) {
  const Shape sh = pick_shape(a.lda, Vec<TA>::V, true);
  // shapes that only columns longer than kMaxM would select are not built
#define SK_CASE(GG, RR)                                                   \
  if constexpr (GG * RR * Vec<TA>::V <= kMaxM) {                          \
    if (sh.G == GG && sh.R == RR) {                                       \
      if constexpr (stream_mode(MODE)) {                                  \
        if (stream) {                                                     \
          launch_one<TA, TC, MODE, GG, RR, true>(a, nblk, st, e0, e1);    \
          return 0;                                                       \
        }                                                                 \
      }                                                                   \
      launch_one<TA, TC, MODE, GG, RR, false>(a, nblk, st, e0, e1);       \
      return 0;                                                           \
    }                                                                     \
  }
  SK_CASE(16, 1) SK_CASE(16, 2) SK_CASE(16, 3) SK_CASE(32, 3)
  SK_CASE(64, 1) SK_CASE(64, 2) SK_CASE(64, 3) SK_CASE(64, 4)
  SK_CASE(64, 6) SK_CASE(64, 8) SK_CASE(64, 12) SK_CASE(64, 16)
#undef SK_CASE
  return -1;
}

template <typename TA, int G, int R>
void launch_sketch_one(const TA* A, int64_t lda, int s, const double* d2, int is_d2,
                       const int32_t* ptr, const int32_t* perm, const int8_t* sign, int w,
                       double* B, int64_t ldb, hipStream_t st) {
  constexpr int NT = 256;
  const int per_block = (NT / 64) * (64 / G);
  int blocks = (w + per_block - 1) / per_block;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_sketch<TA, G, R, NT>), dim3(blocks), dim3(NT), 0, st, A, lda, s, d2,
                     is_d2, ptr, perm, sign, w, B, ldb);
}

template <typename TA>
void sketch_dispatch(const TA* A, int64_t lda, int s, const double* d2, int is_d2,
                     const int32_t* ptr, const int32_t* perm, const int8_t* sign, int w,
                     double* B, int64_t ldb, hipStream_t st) {
  const Shape sh = pick_shape(lda, Vec<TA>::V);
#define SK_CASE(GG, RR)                                                                  \
  if constexpr (GG * RR * Vec<TA>::V <= kMaxM) {                                         \
    if (sh.G == GG && sh.R == RR) {                                                      \
      launch_sketch_one<TA, GG, RR>(A, lda, s, d2, is_d2, ptr, perm, sign, w, B, ldb, st); \
      return;                                                                            \
    }                                                                                    \
  }
  SK_CASE(16, 1) SK_CASE(16, 2)
  SK_CASE(64, 1) SK_CASE(64, 2) SK_CASE(64, 3) SK_CASE(64, 4)
  SK_CASE(64, 6) SK_CASE(64, 8) SK_CASE(64, 12) SK_CASE(64, 16)
#undef SK_CASE
}

}  // namespace

int vec_width(int ta) { return ta == SKIPM_F64 ? 2 : (ta == SKIPM_F32 ? 4 : 8); }

int colpass_nblk_dot(int64_t lda, int64_t n, int ta) {
  const int V = vec_width(ta);
  const Shape sh = pick_shape(lda, V, true);
  if (sh.G == 0) return 1;
  const int64_t slots = (256 / 64) * (64 / sh.G);
  int64_t nb = (n + slots - 1) / slots;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  return (int)nb;
}

int colpass_nblk(int64_t lda, int64_t n, int ta, int tc, int mode) {
  const int V = vec_width(ta);
  const Shape sh = pick_shape(lda, V, true);
  if (sh.G == 0) return 1;
  const int nt = threads_for(mode, sh.R, V, tc == SKIPM_F64 ? 8 : 4, sh.G);
  const int64_t slots = (int64_t)(nt / 64) * (64 / sh.G);
  const int target = nt == 256 ? 512 : 256;
  // at least 16 columns per lane group: fewer, longer workgroups for small
  // matrices, whose passes are bound by each workgroup's fixed start and fold
  // (in the batch engine's grouped launches most of all)
  int64_t nb = (n + slots * 16 - 1) / (slots * 16);
  if (nb > target) nb = target;
  if (nb < 1) nb = 1;
  return (int)nb;
}

int launch_colpass(ColPass& c, hipStream_t st) {
  Args a;
  a.A = c.A;
  a.lda = c.lda;
  a.m = c.m;
  a.n = c.n;
  a.u = c.u;
  a.x = c.x;
  a.s = c.s;
  a.c = c.c;
  a.rd = c.rd;
  a.d2 = c.d2;
  a.rd_out = c.rd_out;
  a.d2_out = c.d2_out;
  a.d2f_out = c.d2f_out;
  a.ds_out = c.ds_out;
  a.t_out = c.t_out;
  a.part = c.part;
  a.ldp = c.ldp;
  a.red = c.red;
  a.sc = c.sc;
  a.done = c.done;
  a.cg = c.cg;
  if (c.nblk <= 0)
    c.nblk = c.mode == COL_DOT ? colpass_nblk_dot(c.lda, c.n, c.ta)
                               : colpass_nblk(c.lda, c.n, c.ta, c.tc, c.mode);
  a.cpb = (c.n + c.nblk - 1) / c.nblk;
  const int nblk = c.nblk;
  int rc = -1;
  if (c.ta == SKIPM_F64 && c.tc == SKIPM_F64) {
    switch (c.mode) {
      case COL_NORMAL:
        rc = dispatch<double, double, COL_NORMAL>(a, nblk, c.nt, st, c.ev0, c.ev1);
        break;
      case COL_PROLOGUE: rc = dispatch<double, double, COL_PROLOGUE>(a, nblk, c.nt, st); break;
      case COL_EPILOGUE: rc = dispatch<double, double, COL_EPILOGUE>(a, nblk, c.nt, st); break;
      case COL_DOT: rc = dispatch<double, double, COL_DOT>(a, nblk, c.nt, st); break;
      case COL_AXPY: rc = dispatch<double, double, COL_AXPY>(a, nblk, c.nt, st); break;
    }
  } else if (c.ta == SKIPM_F32 && c.tc == SKIPM_F64) {
    switch (c.mode) {
      case COL_NORMAL:
        rc = dispatch<float, double, COL_NORMAL>(a, nblk, c.nt, st, c.ev0, c.ev1);
        break;
      case COL_PROLOGUE: rc = dispatch<float, double, COL_PROLOGUE>(a, nblk, c.nt, st); break;
      case COL_EPILOGUE: rc = dispatch<float, double, COL_EPILOGUE>(a, nblk, c.nt, st); break;
      case COL_DOT: rc = dispatch<float, double, COL_DOT>(a, nblk, c.nt, st); break;
    }
  } else if (c.ta == kTypeBF16 && c.tc == SKIPM_F64 && c.mode == COL_NORMAL) {
    // the BF16 copy of A serves the CG products only
    rc = dispatch<bf16_t, double, COL_NORMAL>(a, nblk, c.nt, st, c.ev0, c.ev1);
  }
  return rc;
}

void launch_sketch_dense(const void* A, int ta, int64_t lda, int64_t m, int64_t n, int s,
                         const double* dscale, int is_d2, const int32_t* ptr,
                         const int32_t* perm, const int8_t* sign, int w, double* B,
                         int64_t ldb, hipStream_t st) {
  (void)m;
  (void)n;
  if (ta == SKIPM_F64)
    sketch_dispatch<double>((const double*)A, lda, s, dscale, is_d2, ptr, perm, sign, w, B, ldb,
                            st);
  else
    sketch_dispatch<float>((const float*)A, lda, s, dscale, is_d2, ptr, perm, sign, w, B, ldb,
                           st);
}

int finish_nblk(int64_t m) { return (int)((m + 15) / 16); }

// ---- grouped passes (many matrices of one shape per launch) ----------------

namespace {

Args to_args(const ColPass& c) {
  Args a;
  a.A = c.A;
  a.lda = c.lda;
  a.m = c.m;
  a.n = c.n;
  a.u = c.u;
  a.x = c.x;
  a.s = c.s;
  a.c = c.c;
  a.rd = c.rd;
  a.d2 = c.d2;
  a.rd_out = c.rd_out;
  a.d2_out = c.d2_out;
  a.d2f_out = c.d2f_out;
  a.ds_out = c.ds_out;
  a.t_out = c.t_out;
  a.part = c.part;
  a.ldp = c.ldp;
  a.red = c.red;
  a.sc = c.sc;
  a.done = c.done;
  a.cg = c.cg;
  a.cpb = (c.n + c.nblk - 1) / c.nblk;
  return a;
}

// The lane-group shapes (G, R) of the grouped launches; Args::shape indexes
// this table.
constexpr int kGShapes[][2] = {{16, 1}, {16, 2}, {64, 1},  {64, 2},  {64, 3}, {64, 4},
                               {64, 6}, {64, 8}, {64, 12}, {64, 16}, {32, 3}, {16, 3}};
constexpr int kNGShapes = (int)(sizeof(kGShapes) / sizeof(kGShapes[0]));

// Register class of a shape: the shapes of one launch share its register
// count, the largest that one of them needs, so that shapes of a few
// registers do not run at the occupancy of those of many.
constexpr int gshape_cls(int R) { return R <= 2 ? 0 : (R <= 4 ? 1 : (R <= 8 ? 2 : 3)); }

// Shape i runs in the grouped kernel of block size NT (the block size its own
// launch would take) and register class CLS, for values TA.
template <typename TA, int MODE, int NT, int CLS>
constexpr bool gshape_in(int i) {
  return kGShapes[i][0] * kGShapes[i][1] * Vec<TA>::V <= kMaxM &&
         threads_for(MODE, kGShapes[i][1], Vec<TA>::V, 8, kGShapes[i][0]) == NT &&
         gshape_cls(kGShapes[i][1]) == CLS;
}
template <typename TA, int MODE, int NT, int CLS, int I>
constexpr size_t gshape_lds() {
  if constexpr (gshape_in<TA, MODE, NT, CLS>(I))
    return ColLds<TA, double, kGShapes[I][0], kGShapes[I][1], MODE, NT>::kBytes;
  else
    return 0;
}
template <typename TA, int MODE, int NT, int CLS, int... I>
constexpr size_t gshapes_lds(std::integer_sequence<int, I...>) {
  size_t b = 16;
  ((b = gshape_lds<TA, MODE, NT, CLS, I>() > b ? gshape_lds<TA, MODE, NT, CLS, I>() : b), ...);
  return b;
}

// One pass over several matrices in one launch (the CG of a batch of LPs):
// first[i] is the first workgroup of matrix i (first[nmat] the total), each
// matrix keeps its own lane-group shape, workgroup count, column ranges and
// partials, so its arithmetic is that of its own launch; the matrices of
// every shape whose own launch takes NT threads and that is of register
// class CLS share the launch, and the workgroup's LDS is the largest that
// one of them needs.  Matrix i is at CG
// iteration kstart[i] + j and takes the arguments of that iteration's parity,
// args[2 i + (k & 1)]; a pass outside the CG (kstart null) takes args[i].
template <typename TA, int MODE, int NT, int CLS, bool STREAM>
__global__ __launch_bounds__(NT) void k_colpass_grouped(const Args* __restrict__ args,
                                                        const int32_t* __restrict__ first,
                                                        int nmat,
                                                        const int64_t* __restrict__ kstart,
                                                        int j) {
  int lo = 0, hi = nmat - 1;  // the matrix whose workgroup range holds blockIdx.x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const int64_t k = kstart ? kstart[lo] + j : 0;
  Args a = args[kstart ? 2 * lo + (int)(k & 1) : lo];
  a.cg.k = k;
  const int bid = (int)blockIdx.x - first[lo];
  constexpr size_t kLds =
      gshapes_lds<TA, MODE, NT, CLS>(std::make_integer_sequence<int, kNGShapes>{});
  __shared__ __attribute__((aligned(16))) char smem[kLds];
#define SK_GCASE(I)                                                                      \
  if constexpr (gshape_in<TA, MODE, NT, CLS>(I)) {                                       \
    if (a.shape == I) {                                                                  \
      colpass_body<TA, double, kGShapes[I][0], kGShapes[I][1], MODE, NT, STREAM>(a, bid, \
                                                                                 smem);  \
      return;                                                                            \
    }                                                                                    \
  }
  SK_GCASE(0) SK_GCASE(1) SK_GCASE(2) SK_GCASE(3) SK_GCASE(4) SK_GCASE(5)
  SK_GCASE(6) SK_GCASE(7) SK_GCASE(8) SK_GCASE(9) SK_GCASE(10) SK_GCASE(11)
#undef SK_GCASE
}

template <typename TA, int MODE, int NT, int CLS>
void launch_grouped(const ColKey& k, const Args* args, const int32_t* first, int nmat, int total,
                    const int64_t* kstart, int kit, hipStream_t st) {
  if constexpr (stream_mode(MODE)) {
    if (k.nt) {
      hipLaunchKernelGGL((k_colpass_grouped<TA, MODE, NT, CLS, true>), dim3(total), dim3(NT), 0,
                         st, args, first, nmat, kstart, kit);
      return;
    }
  }
  hipLaunchKernelGGL((k_colpass_grouped<TA, MODE, NT, CLS, false>), dim3(total), dim3(NT), 0, st,
                     args, first, nmat, kstart, kit);
}

template <typename TA, int MODE, int NT>
int dispatch_cls(const ColKey& k, const Args* args, const int32_t* first, int nmat, int total,
                 const int64_t* kstart, int kit, hipStream_t st) {
  switch (k.cls) {
    case 0: launch_grouped<TA, MODE, NT, 0>(k, args, first, nmat, total, kstart, kit, st); return 0;
    case 1: launch_grouped<TA, MODE, NT, 1>(k, args, first, nmat, total, kstart, kit, st); return 0;
    case 2: launch_grouped<TA, MODE, NT, 2>(k, args, first, nmat, total, kstart, kit, st); return 0;
    case 3: launch_grouped<TA, MODE, NT, 3>(k, args, first, nmat, total, kstart, kit, st); return 0;
  }
  return -1;
}

template <typename TA, int MODE>
int dispatch_grouped(const ColKey& k, const Args* args, const int32_t* first, int nmat, int total,
                     const int64_t* kstart, int kit, hipStream_t st) {
  switch (k.threads) {
    case 1024: return dispatch_cls<TA, MODE, 1024>(k, args, first, nmat, total, kstart, kit, st);
    case 768: return dispatch_cls<TA, MODE, 768>(k, args, first, nmat, total, kstart, kit, st);
    case 512: return dispatch_cls<TA, MODE, 512>(k, args, first, nmat, total, kstart, kit, st);
    case 256: return dispatch_cls<TA, MODE, 256>(k, args, first, nmat, total, kstart, kit, st);
  }
  return -1;
}

}  // namespace

size_t colpass_args_bytes() { return sizeof(Args); }

int colpass_prepare(ColPass& c, void* args_out, ColKey* key) {
  if (c.tc != SKIPM_F64 || (c.ta != SKIPM_F64 && c.ta != SKIPM_F32)) return -1;
  if (c.mode != COL_NORMAL && c.mode != COL_DOT) return -1;
  if (c.nblk <= 0)
    c.nblk = c.mode == COL_DOT ? colpass_nblk_dot(c.lda, c.n, c.ta)
                               : colpass_nblk(c.lda, c.n, c.ta, c.tc, c.mode);
  const Shape sh = pick_shape(c.lda, vec_width(c.ta), true);
  int shape = -1;
  for (int i = 0; i < kNGShapes; ++i)
    if (kGShapes[i][0] == sh.G && kGShapes[i][1] == sh.R) shape = i;
  if (shape < 0) return -1;
  key->ta = c.ta;
  key->mode = c.mode;
  key->threads = threads_for(c.mode, sh.R, vec_width(c.ta), 8, sh.G);
  key->cls = gshape_cls(sh.R);
  key->nt = c.mode == COL_NORMAL && c.nt != 0;
  Args a = to_args(c);
  a.shape = shape;
  memcpy(args_out, &a, sizeof(Args));
  return c.nblk;
}

int launch_colpass_grouped(const ColKey& key, const void* dargs, const int32_t* dfirst, int nmat,
                           int total_blocks, const int64_t* kstart, int j, hipStream_t st) {
  const Args* a = (const Args*)dargs;
  if (key.ta == SKIPM_F64)
    return key.mode == COL_NORMAL
               ? dispatch_grouped<double, COL_NORMAL>(key, a, dfirst, nmat, total_blocks, kstart, j,
                                                      st)
               : dispatch_grouped<double, COL_DOT>(key, a, dfirst, nmat, total_blocks, kstart, j, st);
  return key.mode == COL_NORMAL
             ? dispatch_grouped<float, COL_NORMAL>(key, a, dfirst, nmat, total_blocks, kstart, j, st)
             : dispatch_grouped<float, COL_DOT>(key, a, dfirst, nmat, total_blocks, kstart, j, st);
}

void launch_finish_dot_grouped(const FinishDotArgs* dargs, const int32_t* dfirst, int nmat,
                               int total_blocks, const int64_t* kstart, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_dot_grouped, dim3(total_blocks), dim3(256), 0, st, dargs, dfirst,
                     nmat, kstart, j);
}

int launch_finish_dot(const double* part, int64_t ldp, int nblk, int64_t m, const double* dvec,
                      double* out, double* dq_out, const int32_t* done, hipStream_t st) {
  const int blocks = finish_nblk(m);
  hipLaunchKernelGGL(k_finish_dot, dim3(blocks), dim3(256), 0, st, part, ldp, nblk, m, dvec, out,
                     dq_out, done);
  return blocks;
}

void launch_finish(const double* part, int64_t ldp, int64_t off, int nblk, int64_t m,
                   double scale, const double* add, double beta, double* out,
                   const int32_t* done, hipStream_t st) {
  const unsigned blocks = (unsigned)((m + 15) / 16);
  hipLaunchKernelGGL(k_finish<double>, dim3(blocks), dim3(256), 0, st, part, ldp, off, nblk, m,
                     scale, add, beta, out, done);
}

void launch_finish2(const double* part, int64_t ldp, int nblk, int64_t m, int64_t off0,
                    double scale0, const double* add0, double beta0, double* out0, int64_t off1,
                    double scale1, const double* add1, double beta1, double* out1,
                    hipStream_t st) {
  const unsigned blocks = (unsigned)((m + 15) / 16);
  const FinishSet f0{off0, scale0, add0, beta0, out0}, f1{off1, scale1, add1, beta1, out1};
  hipLaunchKernelGGL(k_finish2, dim3(blocks, 2), dim3(256), 0, st, part, ldp, nblk, m, f0, f1);
}

}  // namespace skipm
