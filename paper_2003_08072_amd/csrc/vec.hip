// Vector kernels: fills and copies, the single-workgroup CG state updates, and
// the n-vector passes of one IPM iteration (correction vector and primal
// direction, step length, update).  Every reduction runs in a fixed order
// (per-thread sequential, a fixed DPP sum inside a wave, waves in index
// order, workgroup partials summed in index order), so results are bitwise
// reproducible run to run.
#include <math.h>

#include "common.h"

namespace skipm {

namespace {

constexpr int kVecThreads = 256;
constexpr int kVecBlocksMax = 1024;

__device__ __forceinline__ double wave_sum(double v) { return lane_group_sum<64>(v); }

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over the whole workgroup (result valid in every thread).  `buf` holds
// one slot per wave.
template <int NT>
__device__ double block_sum(double v, double* buf) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) buf[wid] = v;
  __syncthreads();
  double t = 0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) t += buf[q];
  return t;
}

template <int NT>
__device__ double block_min(double v, double* buf) {
  v = wave_min(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) buf[wid] = v;
  __syncthreads();
  double t = INFINITY;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) t = fmin(t, buf[q]);
  return t;
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
// k_fill_f64 that also clears one flag (a factorisation's failure flag)
__global__ void k_fill_f64_flag(double* p, double v, int64_t n, int32_t* flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void k_copy_f64(double* d, const double* s, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = s[i];
}
__global__ void k_cvt_f64_f32(float* d, const double* s, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    d[i] = (float)s[i];
}
template <typename TD, typename TS>
__global__ void k_pad_copy(TD* dst, int64_t ldd, const TS* src, int64_t lds, int64_t m,
                           int64_t n) {
  const int64_t total = ldd * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % ldd, j = e / ldd;
    dst[e] = i < m ? (TD)src[i + j * lds] : (TD)0;
  }
}
// x rounded to bfloat16 (8 significant bits, ties to even), as a 16-bit
// pattern: x is first cut to FP32 by round-to-odd (truncate, then set the
// last bit if anything was cut), which carries enough bits that the final
// round-to-nearest-even to 8 bits equals a direct rounding of x.
__device__ __forceinline__ uint16_t to_bf16(double x) {
  const float t = __double2float_rz(x);
  unsigned b = __float_as_uint(t);
  if ((double)t != x) b |= 1u;
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
template <typename TS>
__global__ void k_pad_copy_bf16(uint16_t* dst, int64_t ldd, const TS* src, int64_t lds, int64_t m,
                                int64_t n) {
  const int64_t total = ldd * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % ldd, j = e / ldd;
    dst[e] = i < m ? to_bf16((double)src[i + j * lds]) : (uint16_t)0;
  }
}
__global__ void k_sqrt(const double* in, double* out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = sqrt(in[i]);
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// ---------------------------------------------------------------------------
// CG state (the iterations themselves are fused into the product and Q^{-1}
// passes, see CgFuse)
//   init:   x = 0, r = rhs, z = P rhs (given), d = z, rz = r^T z,
//           stop threshold tol^2 rz0 (or tol^2 r^T r for the residual test)
//   close:  the bookkeeping of a run stopped by its iteration cap
// The CG kernels return at once when the done flag is set, so a fixed chunk
// of iterations can be enqueued without reading the flag on the host.
// ---------------------------------------------------------------------------
constexpr int kCgThreads = 1024;

__global__ __launch_bounds__(kCgThreads) void k_cg_init(int64_t m, const double* __restrict__ rhs,
                                                        const double* __restrict__ zin,
                                                        double* __restrict__ r,
                                                        double* __restrict__ z,
                                                        double* __restrict__ d,
                                                        float* __restrict__ df,
                                                        double* __restrict__ x,
                                                        double* __restrict__ tw, int64_t nw,
                                                        double* __restrict__ sc,
                                                        int32_t* __restrict__ is, double tol,
                                                        int max_it, int resid_test) {
  __shared__ double buf[kCgThreads / 64];
  double rz = 0, rr = 0;
  for (int64_t i = threadIdx.x; i < m; i += kCgThreads) {
    const double ri = rhs[i], zi = zin[i];
    r[i] = ri;
    z[i] = zi;
    d[i] = zi;
    if (df) df[i] = (float)zi;
    x[i] = 0;
    rz += ri * zi;
    rr += ri * ri;
  }
  for (int64_t i = threadIdx.x; i < nw; i += kCgThreads) tw[i] = 0;
  rz = block_sum<kCgThreads>(rz, buf);
  rr = block_sum<kCgThreads>(rr, buf);
  if (threadIdx.x == 0) {
    sc[S_CG_RZ] = rz;
    sc[S_CG_RZ0] = rz;
    sc[S_CG_RZH0] = rz;
    const double base = resid_test ? rr : rz;
    sc[S_CG_TOL2] = tol > 0 ? tol * tol * base : -1.0;
    sc[S_V_RR] = rr;
    sc[S_V_GG] = rr;
    is[I_CG_ITERS] = 0;
    is[I_CG_MAX] = max_it;
    is[I_CG_DONE] = (max_it <= 0 || !(rz > 0) || (resid_test ? rr : rz) <= sc[S_CG_TOL2]) ? 1 : 0;
    is[I_CG_RESID] = resid_test;
  }
}

// k_cg_init for many LPs, one workgroup each (the same sums in the same order)
__global__ __launch_bounds__(kCgThreads) void k_cg_init_grouped(const CgInitArgs* __restrict__ args) {
  const CgInitArgs& g = args[blockIdx.x];
  __shared__ double buf[kCgThreads / 64];
  double rz = 0, rr = 0;
  for (int64_t i = threadIdx.x; i < g.m; i += kCgThreads) {
    const double ri = g.rhs[i], zi = g.zin[i];
    g.r[i] = ri;
    g.z[i] = zi;
    g.d[i] = zi;
    g.x[i] = 0;
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = block_sum<kCgThreads>(rz, buf);
  rr = block_sum<kCgThreads>(rr, buf);
  if (threadIdx.x == 0) {
    double* sc = g.sc;
    int32_t* is = g.is;
    sc[S_CG_RZ] = rz;
    sc[S_CG_RZ0] = rz;
    sc[S_CG_RZH0] = rz;
    sc[S_CG_TOL2] = g.tol > 0 ? g.tol * g.tol * rz : -1.0;
    sc[S_V_RR] = rr;
    sc[S_V_GG] = rr;
    is[I_CG_ITERS] = 0;
    is[I_CG_MAX] = g.max_it;
    is[I_CG_DONE] = (g.max_it <= 0 || !(rz > 0) || rz <= sc[S_CG_TOL2]) ? 1 : 0;
    is[I_CG_RESID] = 0;
  }
}

// Fused CG stopped by its iteration cap after iteration k - 1: the bookkeeping
// the next iteration's first pass would have done (rz_k, rr_k, count, done).
__global__ __launch_bounds__(64) void k_cg_close(const double* __restrict__ prz, int np,
                                                 int64_t k, double* __restrict__ sc,
                                                 int32_t* __restrict__ is) {
  if (is[I_CG_DONE]) return;
  const int lane = threadIdx.x;
  double s0 = 0, s1 = 0;
  for (int p = lane; p < np; p += 64) {
    s0 += prz[2 * p];
    s1 += prz[2 * p + 1];
  }
  s0 = lane_group_sum<64>(s0);
  s1 = lane_group_sum<64>(s1);
  if (lane == 0) {
    sc[S_CG_RZ] = s0;
    sc[S_V_RR] = s1;
    sc[S_CG_RZH0 + (int)(k & 1)] = s0;
    is[I_CG_ITERS] = (int32_t)k;
    is[I_CG_DONE] = 1;
  }
}

__global__ __launch_bounds__(64) void k_cg_close_grouped(const CgCloseArgs* __restrict__ args,
                                                         int64_t k) {
  const CgCloseArgs& g = args[blockIdx.x];
  if (g.is[I_CG_DONE]) return;
  const int lane = threadIdx.x;
  double s0 = 0, s1 = 0;
  for (int p = lane; p < g.np; p += 64) {
    s0 += g.prz[2 * p];
    s1 += g.prz[2 * p + 1];
  }
  s0 = lane_group_sum<64>(s0);
  s1 = lane_group_sum<64>(s1);
  if (lane == 0) {
    g.sc[S_CG_RZ] = s0;
    g.sc[S_V_RR] = s1;
    g.sc[S_CG_RZH0 + (int)(k & 1)] = s0;
    g.is[I_CG_ITERS] = (int32_t)k;
    g.is[I_CG_DONE] = 1;
  }
}

__global__ __launch_bounds__(256) void k_cg_flags(int32_t* const* __restrict__ is, int nmat,
                                                  int32_t* __restrict__ out) {
  for (int i = threadIdx.x; i < nmat; i += 256) {
    const int32_t* p = is[i];
    out[3 * i] = p[I_CG_DONE];
    out[3 * i + 1] = p[I_CG_ITERS];
    out[3 * i + 2] = p[I_FACT_FAIL];
  }
}

// ---------------------------------------------------------------------------
// IPM n-vector passes
// ---------------------------------------------------------------------------

// ||r_p||^2, b^T y (m-vectors) and the workgroup partials of the prologue
// (||r_d||^2, c^T x, x^T s) -> scalar slots; eta = ||r|| / ||r^0||.
__global__ __launch_bounds__(1024) void k_prologue_finalize(int64_t m, const double* __restrict__ rp,
                                                            const double* __restrict__ b,
                                                            const double* __restrict__ y,
                                                            const double* __restrict__ red,
                                                            int nblk, double* __restrict__ sc,
                                                            int set_origin) {
  __shared__ double buf[16];
  double rp2 = 0, bty = 0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) {
    rp2 += rp[i] * rp[i];
    bty += b[i] * y[i];
  }
  rp2 = block_sum<1024>(rp2, buf);
  bty = block_sum<1024>(bty, buf);
  double rd2 = 0, ctx = 0, xs = 0;
  for (int q = threadIdx.x; q < nblk; q += 1024) {
    rd2 += red[q * 8 + 0];
    ctx += red[q * 8 + 1];
    xs += red[q * 8 + 2];
  }
  rd2 = block_sum<1024>(rd2, buf);
  ctx = block_sum<1024>(ctx, buf);
  xs = block_sum<1024>(xs, buf);
  if (threadIdx.x == 0) {
    sc[S_RP2] = rp2;
    sc[S_BTY] = bty;
    sc[S_RD2] = rd2;
    sc[S_CTX] = ctx;
    const double rn = sqrt(rp2 + rd2);
    if (set_origin) {
      sc[S_R0] = rn;
      sc[S_MU0] = sc[S_MU];
    }
    sc[S_ETA] = sc[S_R0] > 0 ? rn / sc[S_R0] : 0.0;
  }
}

// v_j = sqrt(x_j s_j) sum_r sign_r(j) t[bucket_r(j)]   (eq. compv, t = (ADW)^+ g)
// dx_j = -x_j + sigma mu / s_j - d2_j ds_j - v_j / s_j   (eq. delxhat)
// partials: x^T s, x^T ds + s^T dx, dx^T ds, 1^T v, ||v||^2
__global__ __launch_bounds__(kVecThreads) void k_direction(
    int64_t n, int s, const double* __restrict__ x, const double* __restrict__ sv,
    const double* __restrict__ d2, const double* __restrict__ ds,
    const int32_t* __restrict__ bucket, const int8_t* __restrict__ sign,
    const double* __restrict__ tw, const double* __restrict__ wt, double* __restrict__ v,
    double* __restrict__ dx, double* __restrict__ red, const double* __restrict__ sc) {
  __shared__ double buf[kVecThreads / 64];
  const double smu = sc[S_SIGMA] * sc[S_MU];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = j0 + per < n ? j0 + per : n;
  double a0 = 0, a1 = 0, a2 = 0, vs = 0, v2 = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kVecThreads) {
    const double xj = x[j], sj = sv[j], dsj = ds[j];
    double vj;
    if (wt) {  // Gaussian sketch: wt = (D W_G) t, and sqrt(x_j s_j) / d_j = s_j
      vj = sj * wt[j];
    } else {
      double acc = 0;
      for (int r = 0; r < s; ++r) acc += (double)sign[j * s + r] * tw[bucket[j * s + r]];
      vj = sqrt(xj * sj) * acc;
    }
    const double dxj = -xj + smu / sj - d2[j] * dsj - vj / sj;
    v[j] = vj;
    dx[j] = dxj;
    a0 += xj * sj;
    a1 += xj * dsj + sj * dxj;
    a2 += dxj * dsj;
    vs += vj;
    v2 += vj * vj;
  }
  a0 = block_sum<kVecThreads>(a0, buf);
  a1 = block_sum<kVecThreads>(a1, buf);
  a2 = block_sum<kVecThreads>(a2, buf);
  vs = block_sum<kVecThreads>(vs, buf);
  v2 = block_sum<kVecThreads>(v2, buf);
  if (threadIdx.x == 0) {
    double* o = red + blockIdx.x * 8;
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
    o[3] = vs;
    o[4] = v2;
  }
}

// Smallest alpha >= 0 at which qa a^2 + qb a + qc (qc >= 0) turns negative;
// +inf if never.  Cancellation-free roots: qq = -(qb + sgn(qb) sqrt(disc)) / 2,
// roots qq / qa and qc / qq.
__device__ __forceinline__ double first_exit(double qa, double qb, double qc) {
  if (qc == 0.0) {
    if (qb < 0.0) return 0.0;
    if (qb == 0.0) return qa < 0.0 ? 0.0 : INFINITY;
    return qa < 0.0 ? -qb / qa : INFINITY;
  }
  if (qa == 0.0) return qb < 0.0 ? -qc / qb : INFINITY;
  const double disc = qb * qb - 4.0 * qa * qc;
  if (qa > 0.0) {
    if (qb >= 0.0 || !(disc > 0.0)) return INFINITY;
    const double qq = -0.5 * (qb - sqrt(disc));
    return qc / qq;
  }
  const double sq = sqrt(disc > 0.0 ? disc : 0.0);
  if (qb >= 0.0) {
    const double qq = -0.5 * (qb + sq);
    return qq / qa;
  }
  const double qq = -0.5 * (qb - sq);
  return qc / qq;
}

// Alg. 2 step (e), per entry: first exit of x_i(a) s_i(a) - (1-gamma) mu(a)
// from [0, inf), with n mu(a) = a0 + a1 a + a2 a^2; and the distance to the
// boundary of x, s > 0.  Partials: (min exit, min bound).
__global__ __launch_bounds__(kVecThreads) void k_step_terms(
    int64_t n, const double* __restrict__ x, const double* __restrict__ sv,
    const double* __restrict__ dx, const double* __restrict__ ds, double* __restrict__ red,
    const double* __restrict__ sc) {
  __shared__ double buf[kVecThreads / 64];
  const double g1 = 1.0 - sc[S_GAMMA];
  const double dn = (double)n;
  const double ca = g1 * sc[S_A2] / dn, cb = g1 * sc[S_A1] / dn, cc = g1 * sc[S_A0] / dn;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = j0 + per < n ? j0 + per : n;
  double ex = INFINITY, bd = INFINITY;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kVecThreads) {
    const double xj = x[j], sj = sv[j], dxj = dx[j], dsj = ds[j];
    const double qa = dxj * dsj - ca;
    const double qb = xj * dsj + sj * dxj - cb;
    double qc = xj * sj - cc;
    if (qc < 0.0) qc = 0.0;
    ex = fmin(ex, first_exit(qa, qb, qc));
    if (dxj < 0.0) bd = fmin(bd, -xj / dxj);
    if (dsj < 0.0) bd = fmin(bd, -sj / dsj);
  }
  ex = block_min<kVecThreads>(ex, buf);
  bd = block_min<kVecThreads>(bd, buf);
  if (threadIdx.x == 0) {
    red[blockIdx.x * 8 + 0] = ex;
    red[blockIdx.x * 8 + 1] = bd;
  }
}

// sc[slot0 + q] = sum (op 0) or min (op 1) of red[b*8 + q] over b, q < nq
__global__ __launch_bounds__(1024) void k_reduce_slots(const double* __restrict__ red, int nblk,
                                                       int nq, double* __restrict__ sc, int slot0,
                                                       int op) {
  __shared__ double buf[16];
  for (int q = 0; q < nq; ++q) {
    double v = op ? INFINITY : 0.0;
    for (int b = threadIdx.x; b < nblk; b += 1024)
      v = op ? fmin(v, red[b * 8 + q]) : v + red[b * 8 + q];
    v = op ? block_min<1024>(v, buf) : block_sum<1024>(v, buf);
    if (threadIdx.x == 0) sc[slot0 + q] = v;
  }
}

// Alg. 2 steps (e) and (f) from the reduced terms.
__global__ void k_step_finalize(int64_t n, double* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  const double a0 = sc[S_A0], a1 = sc[S_A1], a2 = sc[S_A2];
  double amax = 1.0;
  amax = fmin(amax, sc[S_EXIT]);
  // residual part of N(gamma): (1 - a) eta <= mu(a) / mu0
  const double t = (double)n * sc[S_MU0] * sc[S_ETA];
  double rc = a0 - t;
  if (rc < 0.0) rc = 0.0;
  amax = fmin(amax, first_exit(a2, a1 + t, rc));
  amax = fmin(amax, (1.0 - sc[S_GUARD]) * sc[S_BOUND]);
  double alpha;
  if (a2 > 0.0) {
    alpha = -a1 / (2.0 * a2);
    if (alpha < 0.0) alpha = 0.0;
    if (alpha > amax) alpha = amax;
  } else {
    alpha = (a1 + a2 * amax <= 0.0) ? amax : 0.0;
  }
  sc[S_AMAX] = amax;
  sc[S_ALPHA] = alpha;
}

// (x, y, s) += alpha (dx, dy, ds) (Alg. 2 step g); partials of the new x^T s.
__global__ __launch_bounds__(kVecThreads) void k_update(
    int64_t n, int64_t m, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ sv, const double* __restrict__ dx, const double* __restrict__ dy,
    const double* __restrict__ ds, double* __restrict__ red, const double* __restrict__ sc) {
  __shared__ double buf[kVecThreads / 64];
  const double alpha = sc[S_ALPHA];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = j0 + per < n ? j0 + per : n;
  double xs = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kVecThreads) {
    const double xj = x[j] + alpha * dx[j];
    const double sj = sv[j] + alpha * ds[j];
    x[j] = xj;
    sv[j] = sj;
    xs += xj * sj;
  }
  if (blockIdx.x == 0)
    for (int64_t i = threadIdx.x; i < m; i += kVecThreads) y[i] += alpha * dy[i];
  xs = block_sum<kVecThreads>(xs, buf);
  if (threadIdx.x == 0) red[blockIdx.x * 8] = xs;
}

__global__ __launch_bounds__(kVecThreads) void k_xs_sum(int64_t n, const double* __restrict__ x,
                                                        const double* __restrict__ sv,
                                                        double* __restrict__ red) {
  __shared__ double buf[kVecThreads / 64];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = j0 + per < n ? j0 + per : n;
  double xs = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kVecThreads) xs += x[j] * sv[j];
  xs = block_sum<kVecThreads>(xs, buf);
  if (threadIdx.x == 0) red[blockIdx.x * 8] = xs;
}

// mu = (sum of partials) / n
__global__ __launch_bounds__(1024) void k_mu_finalize(const double* __restrict__ red, int nblk,
                                                      int64_t n, double* __restrict__ sc) {
  __shared__ double buf[16];
  double v = 0;
  for (int b = threadIdx.x; b < nblk; b += 1024) v += red[b * 8];
  v = block_sum<1024>(v, buf);
  if (threadIdx.x == 0) {
    sc[S_XS] = v;
    sc[S_MU] = v / (double)n;
  }
}

// The whole step tail of Alg. 2 (direction, step length, update, mu) in one
// workgroup, for n <= kVecThreads * 4 where the multi-kernel tail runs one
// workgroup per phase anyway: the same per-entry arithmetic and the same
// workgroup sums in the same order as k_direction, k_step_terms,
// k_step_finalize, k_update and k_mu_finalize, with the one-partial slot
// reductions (exact copies) dropped and six dependent launches saved.
__global__ __launch_bounds__(kVecThreads) void k_step_one(
    int64_t n, int64_t m, int s, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ sv, const double* __restrict__ d2, const double* __restrict__ ds,
    const double* __restrict__ dy, const int32_t* __restrict__ bucket,
    const int8_t* __restrict__ sign, const double* __restrict__ tw,
    const double* __restrict__ wt, double* __restrict__ v, double* __restrict__ dx,
    double* __restrict__ sc) {
  __shared__ double buf[kVecThreads / 64];
  __shared__ double alpha_s;
  const double smu = sc[S_SIGMA] * sc[S_MU];
  double a0 = 0, a1 = 0, a2 = 0, vs = 0, v2 = 0;
  for (int64_t j = threadIdx.x; j < n; j += kVecThreads) {
    const double xj = x[j], sj = sv[j], dsj = ds[j];
    double vj;
    if (wt) {
      vj = sj * wt[j];
    } else {
      double acc = 0;
      for (int r = 0; r < s; ++r) acc += (double)sign[j * s + r] * tw[bucket[j * s + r]];
      vj = sqrt(xj * sj) * acc;
    }
    const double dxj = -xj + smu / sj - d2[j] * dsj - vj / sj;
    v[j] = vj;
    dx[j] = dxj;
    a0 += xj * sj;
    a1 += xj * dsj + sj * dxj;
    a2 += dxj * dsj;
    vs += vj;
    v2 += vj * vj;
  }
  a0 = block_sum<kVecThreads>(a0, buf);
  a1 = block_sum<kVecThreads>(a1, buf);
  a2 = block_sum<kVecThreads>(a2, buf);
  vs = block_sum<kVecThreads>(vs, buf);
  v2 = block_sum<kVecThreads>(v2, buf);
  // step terms (each thread reads back the dx entries it wrote)
  const double g1 = 1.0 - sc[S_GAMMA];
  const double dn = (double)n;
  const double ca = g1 * a2 / dn, cb = g1 * a1 / dn, cc = g1 * a0 / dn;
  double ex = INFINITY, bd = INFINITY;
  for (int64_t j = threadIdx.x; j < n; j += kVecThreads) {
    const double xj = x[j], sj = sv[j], dxj = dx[j], dsj = ds[j];
    const double qa = dxj * dsj - ca;
    const double qb = xj * dsj + sj * dxj - cb;
    double qc = xj * sj - cc;
    if (qc < 0.0) qc = 0.0;
    ex = fmin(ex, first_exit(qa, qb, qc));
    if (dxj < 0.0) bd = fmin(bd, -xj / dxj);
    if (dsj < 0.0) bd = fmin(bd, -sj / dsj);
  }
  ex = block_min<kVecThreads>(ex, buf);
  bd = block_min<kVecThreads>(bd, buf);
  if (threadIdx.x == 0) {
    sc[S_A0] = a0;
    sc[S_A1] = a1;
    sc[S_A2] = a2;
    sc[S_VSUM] = vs;
    sc[S_V2] = v2;
    sc[S_EXIT] = ex;
    sc[S_BOUND] = bd;
    double amax = 1.0;
    amax = fmin(amax, ex);
    const double t = dn * sc[S_MU0] * sc[S_ETA];
    double rc = a0 - t;
    if (rc < 0.0) rc = 0.0;
    amax = fmin(amax, first_exit(a2, a1 + t, rc));
    amax = fmin(amax, (1.0 - sc[S_GUARD]) * bd);
    double alpha;
    if (a2 > 0.0) {
      alpha = -a1 / (2.0 * a2);
      if (alpha < 0.0) alpha = 0.0;
      if (alpha > amax) alpha = amax;
    } else {
      alpha = (a1 + a2 * amax <= 0.0) ? amax : 0.0;
    }
    sc[S_AMAX] = amax;
    sc[S_ALPHA] = alpha;
    alpha_s = alpha;
  }
  __syncthreads();
  const double alpha = alpha_s;
  double xs = 0;
  for (int64_t j = threadIdx.x; j < n; j += kVecThreads) {
    const double xj = x[j] + alpha * dx[j];
    const double sj = sv[j] + alpha * ds[j];
    x[j] = xj;
    sv[j] = sj;
    xs += xj * sj;
  }
  for (int64_t i = threadIdx.x; i < m; i += kVecThreads) y[i] += alpha * dy[i];
  xs = block_sum<kVecThreads>(xs, buf);
  if (threadIdx.x == 0) {
    sc[S_XS] = xs;
    sc[S_MU] = xs / dn;
  }
}

// Start of the correction-vector refinement: t = 0, r = g, ||g||^2 -> slot
// (the sum in k_norm2's order).
__global__ __launch_bounds__(1024) void k_v_init(double* __restrict__ tw, int64_t w,
                                                 double* __restrict__ rv,
                                                 const double* __restrict__ g, int64_t m,
                                                 double* __restrict__ sc, int slot) {
  __shared__ double buf[16];
  for (int64_t i = threadIdx.x; i < w; i += 1024) tw[i] = 0.0;
  double v = 0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) {
    const double gi = g[i];
    rv[i] = gi;
    v += gi * gi;
  }
  v = block_sum<1024>(v, buf);
  if (threadIdx.x == 0) sc[slot] = v;
}

__global__ __launch_bounds__(1024) void k_norm2(const double* __restrict__ u, int64_t m,
                                                double* __restrict__ sc, int slot) {
  __shared__ double buf[16];
  double v = 0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) v += u[i] * u[i];
  v = block_sum<1024>(v, buf);
  if (threadIdx.x == 0) sc[slot] = v;
}

__global__ __launch_bounds__(1024) void k_dot(const double* __restrict__ a,
                                              const double* __restrict__ b, int64_t m,
                                              double* __restrict__ sc, int slot) {
  __shared__ double buf[16];
  double v = 0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) v += a[i] * b[i];
  v = block_sum<1024>(v, buf);
  if (threadIdx.x == 0) sc[slot] = v;
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] += a * x[i];
}

__global__ void k_add(double* __restrict__ out, const double* __restrict__ a,
                      const double* __restrict__ b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = a[i] + b[i];
}

}  // namespace

void launch_add_f64(double* out, const double* a, const double* b, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(256), 0, st, out, a, b, n);
}

void launch_norm2(const double* u, int64_t m, double* sc, int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, st, u, m, sc, slot);
}

void launch_dot(const double* a, const double* b, int64_t m, double* sc, int slot,
                hipStream_t st) {
  hipLaunchKernelGGL(k_dot, dim3(1), dim3(1024), 0, st, a, b, m, sc, slot);
}

void launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, st, y, x, a, n);
}

int vec_nblk(int64_t n) {
  int64_t b = (n + 4 * kVecThreads - 1) / (4 * kVecThreads);
  if (b > kVecBlocksMax) b = kVecBlocksMax;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_fill_f64(double* p, double v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}
void launch_copy_f64(double* dst, const double* src, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(n)), dim3(256), 0, st, dst, src, n);
}
void launch_convert_f64_f32(float* dst, const double* src, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_cvt_f64_f32, dim3(grid_for(n)), dim3(256), 0, st, dst, src, n);
}
void launch_pad_copy_f64(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t m,
                         int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_pad_copy<double, double>), dim3(grid_for(ldd * n)), dim3(256), 0, st, dst,
                     ldd, src, lds, m, n);
}
void launch_pad_copy_f32(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t m,
                         int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_pad_copy<float, float>), dim3(grid_for(ldd * n)), dim3(256), 0, st, dst,
                     ldd, src, lds, m, n);
}
void launch_pad_copy_f64_to_f32(float* dst, int64_t ldd, const double* src, int64_t lds,
                                int64_t m, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_pad_copy<float, double>), dim3(grid_for(ldd * n)), dim3(256), 0, st, dst,
                     ldd, src, lds, m, n);
}
void launch_pad_copy_to_bf16(uint16_t* dst, int64_t ldd, const void* src, int src_dtype,
                             int64_t lds, int64_t m, int64_t n, hipStream_t st) {
  if (src_dtype == SKIPM_F64)
    hipLaunchKernelGGL((k_pad_copy_bf16<double>), dim3(grid_for(ldd * n)), dim3(256), 0, st, dst,
                       ldd, (const double*)src, lds, m, n);
  else
    hipLaunchKernelGGL((k_pad_copy_bf16<float>), dim3(grid_for(ldd * n)), dim3(256), 0, st, dst,
                       ldd, (const float*)src, lds, m, n);
}
void launch_sqrt_vec(int64_t n, const double* in, double* out, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_sqrt, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
}

void launch_cg_init(int64_t m, const double* p, const double* z, double* r, double* zz, double* d,
                    float* df, double* x, double* tw, int64_t nw, double* sc, int32_t* is,
                    double tol, int max_it, int resid_test, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kCgThreads), 0, st, m, p, z, r, zz, d, df, x, tw, nw,
                     sc, is, tol, max_it, resid_test);
}

void launch_cg_close(const double* prz, int np, int64_t k, double* sc, int32_t* is,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_cg_close, dim3(1), dim3(64), 0, st, prz, np, k, sc, is);
}

void launch_cg_init_grouped(const CgInitArgs* dargs, int nmat, hipStream_t st) {
  if (nmat > 0)
    hipLaunchKernelGGL(k_cg_init_grouped, dim3(nmat), dim3(kCgThreads), 0, st, dargs);
}

void launch_cg_close_grouped(const CgCloseArgs* dargs, int nmat, int64_t k, hipStream_t st) {
  if (nmat > 0) hipLaunchKernelGGL(k_cg_close_grouped, dim3(nmat), dim3(64), 0, st, dargs, k);
}

void launch_cg_flags(int32_t* const* is, int nmat, int32_t* out, hipStream_t st) {
  if (nmat > 0) hipLaunchKernelGGL(k_cg_flags, dim3(1), dim3(256), 0, st, is, nmat, out);
}

void launch_prologue_finalize(int64_t m, const double* rp, const double* b, const double* y,
                              const double* red, int nblk, double* sc, int set_origin,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_prologue_finalize, dim3(1), dim3(1024), 0, st, m, rp, b, y, red, nblk, sc,
                     set_origin);
}

void launch_direction(int64_t n, int s, const double* x, const double* sv, const double* d2,
                      const double* ds, const int32_t* bucket, const int8_t* sign,
                      const double* tw, const double* wt, double* v, double* dx, double* red,
                      int nblk, const double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_direction, dim3(nblk), dim3(kVecThreads), 0, st, n, s, x, sv, d2, ds,
                     bucket, sign, tw, wt, v, dx, red, sc);
}

void launch_reduce_slots(const double* red, int nblk, int nq, double* sc, int slot0, int op,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_slots, dim3(1), dim3(1024), 0, st, red, nblk, nq, sc, slot0, op);
}

void launch_step_terms(int64_t n, const double* x, const double* s, const double* dx,
                       const double* ds, double* red, int nblk, const double* sc,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_step_terms, dim3(nblk), dim3(kVecThreads), 0, st, n, x, s, dx, ds, red, sc);
}

void launch_step_finalize(int64_t n, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_step_finalize, dim3(1), dim3(64), 0, st, n, sc);
}

void launch_update(int64_t n, int64_t m, double* x, double* y, double* s, const double* dx,
                   const double* dy, const double* ds, double* red, int nblk, const double* sc,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3(nblk), dim3(kVecThreads), 0, st, n, m, x, y, s, dx, dy, ds,
                     red, sc);
}

void launch_xs_sum(int64_t n, const double* x, const double* s, double* red, int nblk,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_xs_sum, dim3(nblk), dim3(kVecThreads), 0, st, n, x, s, red);
}

void launch_step_one(int64_t n, int64_t m, int s, double* x, double* y, double* sv,
                     const double* d2, const double* ds, const double* dy, const int32_t* bucket,
                     const int8_t* sign, const double* tw, const double* wt, double* v,
                     double* dx, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_step_one, dim3(1), dim3(kVecThreads), 0, st, n, m, s, x, y, sv, d2, ds,
                     dy, bucket, sign, tw, wt, v, dx, sc);
}

void launch_fill_f64_flag(double* p, double v, int64_t n, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f64_flag, dim3(grid_for(n)), dim3(256), 0, st, p, v, n, flag);
}

void launch_v_init(double* tw, int64_t w, double* rv, const double* g, int64_t m, double* sc,
                   int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_v_init, dim3(1), dim3(1024), 0, st, tw, w, rv, g, m, sc, slot);
}

void launch_mu_finalize(const double* red, int nblk, int64_t n, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_mu_finalize, dim3(1), dim3(1024), 0, st, red, nblk, n, sc);
}

}  // namespace skipm
