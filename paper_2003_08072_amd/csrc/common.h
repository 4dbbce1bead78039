// Internal declarations shared by the HIP translation units of libskipm.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>

#include <string>

#include "../../include/skipm.h"

namespace skipm {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

#define SK_CHECK_HIP(expr)                                                         \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::skipm::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      return SKIPM_EDEVICE;                                                        \
    }                                                                              \
  } while (0)

#define SK_TRY(expr)                  \
  do {                                \
    int rc_ = (expr);                 \
    if (rc_ != SKIPM_OK) return rc_;  \
  } while (0)

constexpr int kWave = 64;
// element type of a low-precision copy of A (alongside SKIPM_F64 / SKIPM_F32):
// bfloat16, rounded to nearest even
constexpr int kTypeBF16 = 2;
// Largest m (rows of A) the library takes: the column passes keep a column of
// up to this many rows in one lane group's registers, the sparse passes keep
// an m-vector in LDS.
constexpr int64_t kMaxM = 2048;

// ---------------------------------------------------------------------------
// Sum of an FP64 value over a lane group of G = 16 (a DPP row), 32 (half
// the wave) or 64 (the wave) lanes, the same bits in every lane of the group:
// pairs of lanes (xor 1, xor 2 by quad permutes), then the two halves of each
// 8-lane half row and of each 16-lane row (mirrors: lane i against 7 - i,
// 15 - i), each by DPP moves of the two 32-bit halves; then the four rows'
// sums read from lanes 0, 16, 32, 48 and added as r0 + r1, r2 + r3 (halves)
// or (r0 + r1) + (r2 + r3) (the wave).  No LDS permute, so the chain is a few
// cycles per step.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
template <int G>
__device__ __forceinline__ double lane_group_sum(double v) {
  static_assert(G == 16 || G == 32 || G == 64, "lane groups of 16, 32 or 64 lanes");
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane xor 1
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane xor 2
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  if constexpr (G == 64) {
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    v = (r0 + r1) + (r2 + r3);
  } else if constexpr (G == 32) {
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    v = (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
  }
  return v;
}
// A pass over A streams it with non-temporal loads once A takes most of the
// 256 MiB Infinity Cache (240 MiB: measured, 200.8 MB read 16 % faster
// cached, 263 MB 1.6 % faster streamed); a smaller one stays cached.
constexpr int64_t kStreamBytes = (int64_t)240 << 20;

// ---------------------------------------------------------------------------
// device scalar slots (one FP64 array per handle)
// ---------------------------------------------------------------------------
enum Slot : int {
  S_MU = 0,      // x^T s / n of the current iterate
  S_XS,          // x^T s
  S_CTX,         // c^T x
  S_BTY,         // b^T y
  S_RP2,         // ||r_p||^2
  S_RD2,         // ||r_d||^2
  S_A0, S_A1, S_A2,  // step sums x^T s, x^T ds + s^T dx, dx^T ds
  S_VSUM, S_V2,  // 1^T v, ||v||^2
  S_AMAX, S_ALPHA,
  S_ETA,         // ||r^k|| / ||r^0||
  S_MU0,         // mu of the origin
  S_R0,          // ||r^0||
  S_SIGMA, S_GAMMA, S_GUARD,
  S_EXIT,        // min first-exit over the per-entry conditions
  S_BOUND,       // distance to the boundary of x, s > 0
  // CG state
  S_CG_RZ, S_CG_RZ0, S_CG_TOL2, S_CG_PQ,
  S_V_RR, S_V_GG, // v-solve: ||r||^2, ||g||^2
  S_RHO2,         // mixed precision: r^T Q^{-1} r of the FP64 normal-equation residual
  S_CG_RZH0, S_CG_RZH1,  // fused CG: r_k^T z_k of iteration k in slot S_CG_RZH0 + k % 2
  S_NSLOTS = 40
};

enum IntSlot : int {
  I_CG_ITERS = 0,   // iterations performed by the running CG
  I_CG_DONE,        // 1: converged (or broke down); later CG kernels return at once
  I_CG_MAX,         // iteration cap of the running CG
  I_FACT_FAIL,      // non-positive pivot met while inverting the Gram matrix
  I_CG_RESID,       // 1: stop on the residual r^T r, 0: on r^T z
  I_NINTS = 8
};

// ---------------------------------------------------------------------------
// kernel launchers (each defined in the .hip file that owns the kernel)
// ---------------------------------------------------------------------------

// fill / copy helpers
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t st);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
void launch_copy_f64(double* dst, const double* src, int64_t n, hipStream_t st);
void launch_convert_f64_f32(float* dst, const double* src, int64_t n, hipStream_t st);
void launch_pad_copy_f64(double* dst, int64_t ldd, const double* src, int64_t lds,
                         int64_t m, int64_t n, hipStream_t st);
void launch_pad_copy_f32(float* dst, int64_t ldd, const float* src, int64_t lds,
                         int64_t m, int64_t n, hipStream_t st);
void launch_pad_copy_f64_to_f32(float* dst, int64_t ldd, const double* src, int64_t lds,
                                int64_t m, int64_t n, hipStream_t st);
// bfloat16 copy (round to nearest even, from FP64 or FP32 source values)
void launch_pad_copy_to_bf16(uint16_t* dst, int64_t ldd, const void* src, int src_dtype,
                             int64_t lds, int64_t m, int64_t n, hipStream_t st);

// hash + counting sort of (row, block) items by bucket
void launch_hash(uint64_t seed, int64_t k, int s, int64_t n, int w, int32_t* bucket,
                 int8_t* sign, int32_t* count, hipStream_t st);
void launch_bucket_scan(const int32_t* count, int32_t* ptr, int32_t* cursor, int w,
                        hipStream_t st);
// w: the number of buckets (at most 8192 takes the LDS-aggregated kernel)
void launch_bucket_scatter(const int32_t* bucket, int64_t nitems, int w, const int32_t* ptr,
                           int32_t* cursor, int32_t* perm, hipStream_t st);
void launch_bucket_sort(const int32_t* ptr, const int32_t* raw, int32_t* perm, int w,
                        hipStream_t st);

// dense column passes
// CG bookkeeping fused into the passes of one preconditioned CG iteration k
// (M = Q, z = Q^{-1} r):
//   COL_NORMAL pass:  rz_k, rr_k from the previous COL_DOT pass's partials;
//                     stop test; beta_k = rz_k / rz_{k-1}; d_k = z_k + beta_k d_{k-1}
//                     (every block forms d_k for itself, block 0 stores it);
//                     then q_k = A D^2 A^T d_k as usual
//   finish:           q_k, and per-block partials of d_k^T q_k
//   COL_DOT over Q^{-1}: alpha_k = rz_k / d_k^T q_k; w = Q^{-1} q_k; x += alpha d;
//                     r -= alpha q; z -= alpha w; per-block partials of r^T z, r^T r
// Every partial is summed in a fixed order, so the iterates are reproducible.
struct CgFuse {
  int on = 0;
  int inner = SKIPM_INNER_CG;  // CG: beta_k = rz_k / rz_{k-1}; SD: beta = 0;
                               // Richardson: beta = 0 and alpha = 1
  int64_t k = 0;               // CG iteration
  const double* z = nullptr;   // NORMAL: z_k
  const double* d_old = nullptr;  // NORMAL: d_{k-1} (d_0 itself when k = 0)
  double* d_new = nullptr;     // NORMAL: d_k (written by block 0)
  const double* prz = nullptr; // NORMAL: [np][2] partial (r^T z, r^T r)
  int np = 0;
  double* sc = nullptr;
  int32_t* is = nullptr;
  const double* q = nullptr;   // DOT: q_k
  const double* d = nullptr;   // DOT: d_k
  double* x = nullptr;         // DOT: the CG solution
  double* r = nullptr;
  double* zz = nullptr;
  const double* pdq = nullptr; // DOT: [nf] partial d^T q of the finish
  int nf = 0;
  double* prz_out = nullptr;   // DOT: [nblk][2]
};

struct ColPass {
  int mode;                 // see COL_* below
  const void* A;            // column-major, element type ta
  int ta;                   // SKIPM_F64 / SKIPM_F32
  int tc;                   // accumulation type: SKIPM_F64 (the only one built)
  int64_t lda, m, n;
  const void* u;            // m-vector (type tc) for the column dots
  const double* x;          // per-column inputs (FP64)
  const double* s;
  const double* c;
  const double* rd;
  const void* d2;           // column scale (type tc), NULL = 1; COL_AXPY: the coefficients
  double* rd_out;
  double* d2_out;
  float* d2f_out;
  double* ds_out;
  void* t_out;              // per-column dot a_j^T u (type tc)
  void* part;               // [nblk][nacc*ldp] partial sums (type tc)
  int64_t ldp;
  double* red;              // [nblk][8] partial scalars (prologue)
  const double* sc;         // device scalar slots
  const int32_t* done;      // optional early-exit flag
  int nblk;                 // filled by the launcher
  int nt = 0;               // NORMAL/PROLOGUE/EPILOGUE over an A that takes most of the
                            // Infinity Cache: non-temporal column loads
  CgFuse cg;                // fused CG bookkeeping (COL_NORMAL, COL_DOT)
  hipEvent_t ev0 = nullptr;  // COL_NORMAL: optional events stamped with the kernel's
  hipEvent_t ev1 = nullptr;  // start and end (sampled timing)
};
enum { COL_NORMAL = 0, COL_PROLOGUE = 1, COL_EPILOGUE = 2, COL_DOT = 3, COL_AXPY = 4 };
int launch_colpass(ColPass& a, hipStream_t st);

// Grouped passes: the CG passes of many LPs in one launch per pass, block
// size and register class; each matrix keeps its own lane-group shape,
// carried in its argument block.  colpass_prepare fills the kernel arguments of one pass
// (colpass_args_bytes() bytes, to be copied to the device) and the launch
// key; returns its workgroup count, or -1 for a pass the grouped kernels do
// not cover (only COL_NORMAL and COL_DOT over FP64 / FP32 values).  Passes
// launched together must share the key.
struct ColKey {
  int ta = 0, mode = 0, threads = 0, cls = 0;
  bool nt = false;
  bool operator==(const ColKey& o) const {
    return ta == o.ta && mode == o.mode && threads == o.threads && cls == o.cls && nt == o.nt;
  }
};
size_t colpass_args_bytes();
int colpass_prepare(ColPass& c, void* args_out, ColKey* key);
// dargs: the argument blocks (two per matrix, for even and odd CG iterations,
// when kstart is given: matrix i is at iteration kstart[i] + j; else one);
// dfirst: nmat + 1 workgroup offsets (device)
int launch_colpass_grouped(const ColKey& key, const void* dargs, const int32_t* dfirst, int nmat,
                           int total_blocks, const int64_t* kstart, int j, hipStream_t st);
struct FinishDotArgs {
  const double* part;
  int64_t ldp;
  int nblk;
  int64_t m;
  const double* dvec;
  double* out;
  double* dq_out;
  const int32_t* done;
};
// dargs: two per LP (even, odd iteration); LP i at iteration kstart[i] + j
void launch_finish_dot_grouped(const FinishDotArgs* dargs, const int32_t* dfirst, int nmat,
                               int total_blocks, const int64_t* kstart, int j, hipStream_t st);
// the CG bookkeeping kernels, one workgroup per LP
struct CgInitArgs {
  int64_t m;
  const double* rhs;
  const double* zin;
  double *r, *z, *d, *x;
  double* sc;
  int32_t* is;
  double tol;
  int max_it;
};
void launch_cg_init_grouped(const CgInitArgs* dargs, int nmat, hipStream_t st);
struct CgCloseArgs {
  const double* prz;
  int np;
  double* sc;
  int32_t* is;
};
void launch_cg_close_grouped(const CgCloseArgs* dargs, int nmat, int64_t k, hipStream_t st);
// out[3 i .. 3 i + 2] = (done, iterations, factorisation failure) of LP i
void launch_cg_flags(int32_t* const* is, int nmat, int32_t* out, hipStream_t st);

// A whole CG solve in one workgroup (small dense LPs): A (lda x n, element
// type given to the launcher), D^2 (n), Q^{-1} (mp x mp), right-hand side
// (m); the solution goes to x, the final r, z, d to r, z, d (each may be
// null), the scalars and counters to the same slots as the fused CG.
struct SmallCg {
  const void* A = nullptr;
  int64_t lda = 0, m = 0, n = 0;
  const double* d2 = nullptr;
  const double* Qi = nullptr;
  int64_t mp = 0;
  const double* rhs = nullptr;
  double* x = nullptr;
  double* r = nullptr;
  double* z = nullptr;
  double* d = nullptr;
  double* sc = nullptr;
  int32_t* is = nullptr;
  double tol = 0;
  int max_it = 0;
  int inner = SKIPM_INNER_CG;
};
// Returns -1 (and launches nothing) for shapes it does not cover.
int launch_cg_small(const SmallCg& a, int ta, hipStream_t st);
// workgroups of a pass (each writes one partial of nacc * m entries)
int colpass_nblk(int64_t lda, int64_t n, int ta, int tc, int mode);

// bucket-ordered sketch B[:, b] = sum over items in bucket b of sign * d_j * A[:, j]
// (dscale holds d, or d^2 when is_d2 != 0)
// Gaussian sketch (dense A): Wd = D W_G, n x w column-major with leading dim ldw
void launch_gauss_fill(uint64_t seed, int64_t k, int64_t n, int64_t w, const double* dscale,
                       int is_d2, double* Wd, int64_t ldw, hipStream_t st);
// out[i] = sum over the ns slices part[s lw + i] (fixed order)
void launch_sum_slices(const double* part, int ns, int64_t lw, double* out, hipStream_t st);
// K-split of the Gaussian sketch GEMM: number of slices for m x w x n
int gauss_ksplit(int64_t lda, int64_t w, int64_t n);
// B_s = A[:, slice s] Wd[slice s, :] on the FP64 matrix cores for the slices
// of n that gauss_gemm_slices(n, ns) counts (out: that many lda x w blocks;
// with one slice, out is B itself); Wd has leading dimension ldw (even)
void launch_gauss_gemm(const double* A, int64_t lda, const double* Wd, int64_t ldw, int64_t w,
                       int64_t n, int ns, double* out, hipStream_t st);
int gauss_gemm_slices(int64_t n, int ns);
// gy = Wd t (n rows, w columns)
void launch_gauss_gemv(const double* Wd, int64_t ldw, int64_t n, int64_t w, const double* t,
                       double* gy, hipStream_t st);
void launch_sketch_dense(const void* A, int ta, int64_t lda, int64_t m, int64_t n, int s,
                         const double* dscale, int is_d2, const int32_t* ptr,
                         const int32_t* perm, const int8_t* sign, int w, double* B,
                         int64_t ldb, hipStream_t st);

// sum of partials along the block axis: out[i] = scale*sum_b part[b][off+i] + beta*add[i]
// launch_finish plus, per workgroup of 16 rows, the partial sum of dvec_i out_i
// (dq_out[blockIdx]); returns the number of workgroups
int launch_finish_dot(const double* part, int64_t ldp, int nblk, int64_t m, const double* dvec,
                      double* out, double* dq_out, const int32_t* done, hipStream_t st);
int finish_nblk(int64_t m);
int colpass_nblk_dot(int64_t lda, int64_t n, int ta);
void launch_finish(const double* part, int64_t ldp, int64_t off, int nblk, int64_t m,
                   double scale, const double* add, double beta, double* out,
                   const int32_t* done, hipStream_t st);
// two launch_finish of the same partials (offsets off0 and off1) in one launch
void launch_finish2(const double* part, int64_t ldp, int nblk, int64_t m, int64_t off0,
                    double scale0, const double* add0, double beta0, double* out0, int64_t off1,
                    double scale1, const double* add1, double beta1, double* out1,
                    hipStream_t st);

// sparse A: CSR for products A v (rows cut into segments of at most kSeg
// non-zeros), CSC for the column dots and the sketch
struct SparseA {
  int64_t m = 0, n = 0, nnz = 0;
  int vdt = SKIPM_F64;
  const int32_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
  const void* val = nullptr;
  const int32_t* colptr = nullptr;
  const int32_t* rowidx = nullptr;
  const void* cval = nullptr;
  int64_t nseg = 0;
  const int32_t* segptr = nullptr;
  const int32_t* seg_start = nullptr;
  const int32_t* seg_end = nullptr;
  // column blocks of the one-pass normal product: bdesc[4 b ..] = (first
  // column, columns, non-zeros, first slot) of block b; its slots of the
  // keyed copy of its non-zeros in column order (ck = local column << 16 |
  // row, cv), and their (row, column) order: FP64 values as a second keyed
  // copy (rk = row << 16 | local column, rv), FP32 values as 16-bit references
  // (rp: the block-local slot of the column-order entry, bits 13 and 14 marking
  // the row's first and last non-zero).  Bits 12 and 13 of a key mark its
  // column's (row's) first and last non-zero.
  int64_t nbk = 0;
  const int32_t* bdesc = nullptr;
  const uint32_t* ck = nullptr;
  const void* cv = nullptr;
  const uint32_t* rk = nullptr;
  const void* rv = nullptr;
  const uint16_t* rp = nullptr;
};
constexpr int kSeg = 512;
// One-pass sparse normal product (column blocks, LDS coefficients).
// sb_partition cuts the columns into blocks and lays out their slots (host
// vector of 4 nbk block descriptors; returns the slot count, or -1 on a HIP
// error); sb_fill (A->nbk set, bdesc on the device) writes the column-order
// copy and the row order (rk, rv for FP64 values, rp for FP32; the others
// null) and records them in A; bad |= 4 if a block broke its bounds.
int64_t sb_partition(const SparseA& A, std::vector<int32_t>* bdesc, hipStream_t st);
void sb_fill(SparseA* A, const int32_t* bdesc, uint32_t* ck, void* cv, uint32_t* rk, void* rv,
             uint16_t* rp, int32_t* bad, hipStream_t st);
int64_t sb_max_blocks(int64_t n, int64_t nnz);  // upper bounds: block count,
int64_t sb_max_slots(int64_t n, int64_t nnz);   // slots of each keyed copy
// part[b][i] (b < A.nbk, leading dimension ldp >= m) = sum over block b's
// columns j of a_ij c_j (a_j^T u) (c null: c_j = 1).  With cg, the pass opens
// a CG iteration as the dense product pass does (u is then d_0 at k = 0).
int launch_sb_normal(const SparseA& A, const double* u, const double* c, double* part,
                     int64_t ldp, const int32_t* done, hipStream_t st, const CgFuse* cg = nullptr);
void launch_csr_check(const int32_t* rowptr, const int32_t* colidx, int64_t m, int64_t n,
                      int64_t nnz, int32_t* bad, hipStream_t st);
void launch_build_csc(const int32_t* rowptr, const int32_t* colidx, const void* val, int vdt,
                      int64_t m, int64_t n, int64_t nnz, int32_t* cnt, int32_t* colptr,
                      int32_t* cursor, int32_t* rowidx, void* cval, hipStream_t st);
void launch_build_segments(const int32_t* rowptr, int64_t m, int seg, int32_t* nseg,
                           int32_t* segptr, int32_t* cursor, int32_t* seg_start, int32_t* seg_end,
                           hipStream_t st);
// per column j: t_j = a_j^T u and the mode's work (COL_NORMAL: coef1 = d2 t;
// COL_PROLOGUE: r_d, d^2, coef2 = sigma mu / s + d^2 r_d; COL_EPILOGUE: ds,
// coef1 = d2 t; COL_DOT: coef1 = t)
int launch_csc_dot(const SparseA& A, int mode, const double* u, const double* x, const double* s,
                   const double* c, const double* rd, const double* d2, double* coef1,
                   double* coef2, double* rd_out, double* d2_out, double* ds_out, double* red,
                   const double* sc, const int32_t* done, int nblk, hipStream_t st,
                   const CgFuse* cg = nullptr);
int csc_dot_nblk(int64_t n);
int csr_fold_nblk(int64_t m);
// segment sums of A coef1 (and A coef2), then out = scale * (A coef_which) + beta * add
void launch_csr_segsum(const SparseA& A, const double* coef1, const double* coef2,
                       double* segsum, const int32_t* done, hipStream_t st);
void launch_csr_fold(const SparseA& A, const double* segsum, int which, double scale,
                     const double* add, double beta, double* out, const int32_t* done,
                     hipStream_t st, const double* dvec = nullptr, double* dq_out = nullptr);
void launch_sketch_csc(const SparseA& A, int s, const double* dscale, int is_d2,
                       const int32_t* ptr, const int32_t* perm, const int8_t* sign, int w,
                       double* B, int64_t ldb, hipStream_t st);

// Gram matrix and its inverse (blocked Cholesky, triangular inverse, X^T X)
int gram_ksplit(int64_t mp, int64_t w);  // column splits of the Gram (launch_gram)
void launch_gram(const double* B, int64_t ldb, int64_t m, int64_t w, double* Gpart,
                 int ksplit, int64_t mp, hipStream_t st);
void launch_gram_finish(const double* Gpart, int ksplit, int64_t m, int64_t mp, double* G,
                        hipStream_t st);
// G (mp x mp, SPD, mp a multiple of 64) -> G^{-1} in place via Cholesky; Xb: mp x mp
// (holds L^{-1}), Ct: mp x mp scratch
void launch_spd_inverse(double* G, double* Xb, double* Ct, int64_t mp, int32_t* fail,
                        hipStream_t st);
void launch_shift_diag(double* G, int64_t mp, int64_t m, double rel, hipStream_t st);
// Out = X In, X block-lower-triangular mp x mp
void launch_trmm(const double* X, int64_t mp, const double* In, int64_t ldin, int64_t nrows,
                 int64_t ncols, double* Out, int64_t ldout, int64_t nrows_out, hipStream_t st);
void launch_shift_trace(double* G, int64_t mp, int64_t m, double c, hipStream_t st);
// sc[slot] = ||u||^2 over m entries (single workgroup)
void launch_norm2(const double* u, int64_t m, double* sc, int slot, hipStream_t st);
void launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st);
// out = a + b (n entries)
void launch_add_f64(double* out, const double* a, const double* b, int64_t n, hipStream_t st);
// sc[slot] = a^T b over m entries (single workgroup)
void launch_dot(const double* a, const double* b, int64_t m, double* sc, int slot,
                hipStream_t st);

// single-workgroup CG kernels
void launch_cg_init(int64_t m, const double* p, const double* z, double* r, double* zz,
                    double* d, float* df, double* x, double* tw, int64_t nw, double* sc,
                    int32_t* is, double tol, int max_it, int resid_test, hipStream_t st);
// fused CG: close a run stopped by its iteration cap after iteration k - 1
// (rz_k, rr_k from the partials, iteration count k, done flag)
void launch_cg_close(const double* prz, int np, int64_t k, double* sc, int32_t* is,
                     hipStream_t st);

// n-vector kernels of the IPM iteration
void launch_prologue_finalize(int64_t m, const double* rp, const double* b, const double* y,
                              const double* red, int nblk, double* sc, int set_origin,
                              hipStream_t st);
void launch_mu_finalize(const double* red, int nblk, int64_t n, double* sc, hipStream_t st);
void launch_direction(int64_t n, int s, const double* x, const double* sv, const double* d2,
                      const double* ds, const int32_t* bucket, const int8_t* sign,
                      const double* tw, const double* wt, double* v, double* dx, double* red,
                      int nblk, const double* sc, hipStream_t st);
void launch_reduce_slots(const double* red, int nblk, int nq, double* sc, int slot0,
                         int op, hipStream_t st);
void launch_step_terms(int64_t n, const double* x, const double* s, const double* dx,
                       const double* ds, double* red, int nblk, const double* sc,
                       hipStream_t st);
void launch_step_finalize(int64_t n, double* sc, hipStream_t st);
void launch_update(int64_t n, int64_t m, double* x, double* y, double* s, const double* dx,
                   const double* dy, const double* ds, double* red, int nblk,
                   const double* sc, hipStream_t st);
void launch_xs_sum(int64_t n, const double* x, const double* s, double* red, int nblk,
                   hipStream_t st);
void launch_sqrt_vec(int64_t n, const double* in, double* out, hipStream_t st);
int vec_nblk(int64_t n);
// p[0..n) = v and *flag = 0 in one launch.
void launch_fill_f64_flag(double* p, double v, int64_t n, int32_t* flag, hipStream_t st);
// tw[0..w) = 0, rv = g (m entries), sc[slot] = ||g||^2.
void launch_v_init(double* tw, int64_t w, double* rv, const double* g, int64_t m, double* sc,
                   int slot, hipStream_t st);
// One-workgroup step tail (direction, step length, update, mu) for
// vec_nblk(n) == 1; same results as the multi-kernel tail.
void launch_step_one(int64_t n, int64_t m, int s, double* x, double* y, double* sv,
                     const double* d2, const double* ds, const double* dy, const int32_t* bucket,
                     const int8_t* sign, const double* tw, const double* wt, double* v,
                     double* dx, double* sc, hipStream_t st);

}  // namespace skipm
