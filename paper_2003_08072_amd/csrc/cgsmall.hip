// Whole CG solves of small LPs in one workgroup (Alg. 1 step 3 with M = Q, the
// same iteration as the fused multi-launch CG).
//
// When A (FP64) fits comfortably in one XCD's L2 and m <= 64, a CG iteration is a few microseconds of work, and the launches,
// the partial-sum folds and the host's chunk checks of the multi-workgroup
// path cost several times more than the work.  Here one workgroup of 1024
// threads runs every iteration: the product q = A D^2 A^T d (one pass over A,
// a lane group per column as in the column pass), d^T q, w = Q^{-1} q (a pass
// over the columns of Q^{-1}), the x, r, z updates and the next r^T z, r^T r,
// with the m-vectors in LDS and __syncthreads between the phases.  Every sum
// is taken in a fixed order, so results are bitwise reproducible.
#include "common.h"

namespace skipm {

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));

template <typename TA>
struct SVec;
template <>
struct SVec<double> {
  static constexpr int V = 2;
  typedef dv2 type;
};

constexpr int kNT = 1024;
constexpr int kNW = kNT / 64;

template <int G>
__device__ __forceinline__ double gsum(double v) {
  return lane_group_sum<G>(v);
}

// Sum over the workgroup in a fixed order (fixed sum per wave, waves in
// order); every thread returns the total.
__device__ __forceinline__ void block_sum2(double& a, double& b, double (*red)[2], int lane,
                                           int wid) {
  a = lane_group_sum<64>(a);
  b = lane_group_sum<64>(b);
  __syncthreads();  // red may still be read from the previous use
  if (lane == 0) {
    red[wid][0] = a;
    red[wid][1] = b;
  }
  __syncthreads();
  double s0 = 0, s1 = 0;
  for (int w = 0; w < kNW; ++w) {
    s0 += red[w][0];
    s1 += red[w][1];
  }
  a = s0;
  b = s1;
}

// A: G lanes per column, R vectors of V rows per lane (rows (r G + lg) V + e).
// Q^{-1}: GQ lanes per column, RQ vectors of 2 rows per lane.
template <typename TA, int G, int R, int GQ, int RQ>
__global__ __launch_bounds__(kNT) void k_cg_small(SmallCg a) {
  constexpr int V = SVec<TA>::V;
  // columns per chunk (two chunks of CH R vectors in registers; at R = 2 this
  // passes 128 VGPRs by a few spilled ones and still measured faster than one
  // column per chunk: config 0 52.8 -> 53.3 solves/s, the same sums)
  constexpr int CH = 2;
  typedef typename SVec<TA>::type VT;
  constexpr int LROWS = G * R * V;
  constexpr int LQ = GQ * RQ * 2;
  constexpr int LV = LQ > LROWS ? LQ : LROWS;
  constexpr int NGW = 64 / G, NSLOT = kNW * NGW;
  constexpr int NGWQ = 64 / GQ, NSLOTQ = kNW * NGWQ;
  __shared__ double sx[LV], sr[LV], sz[LV], sd[LV], sq[LV];
  __shared__ double wbuf[kNW * LROWS];
  __shared__ double red[kNW][2];

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = lane / G, lg = lane % G;
  const int slot = wid * NGW + grp;
  const int grpq = lane / GQ, lgq = lane % GQ;
  const int slotq = wid * NGWQ + grpq;
  const int64_t m = a.m, n = a.n;
  const TA* __restrict__ A = (const TA*)a.A;
  const double* __restrict__ Qi = a.Qi;

  bool valid[R];
  int vrow[R];    // vector index read for row vector r (0 when past lda)
  VT vmask[R];    // 1 for rows within lda, 0 past it
#pragma unroll
  for (int r = 0; r < R; ++r) {
    valid[r] = (int64_t)(r * G + lg) * V < a.lda;
    vrow[r] = valid[r] ? r * G + lg : 0;
    vmask[r] = (VT)(valid[r] ? 1 : 0);
  }
  bool validq[RQ];
#pragma unroll
  for (int r = 0; r < RQ; ++r) validq[r] = (int64_t)(r * GQ + lgq) * 2 < a.mp;

  // w_j = (Q^{-1} u)_j for the columns j < m this lane group owns, then
  // f(j, w_j) on lane 0 of the group
  auto qpass = [&](const double* u, auto&& f) {
    double uq[RQ][2];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const int row0 = (r * GQ + lgq) * 2;
      uq[r][0] = validq[r] ? u[row0] : 0.0;
      uq[r][1] = validq[r] ? u[row0 + 1] : 0.0;
    }
    for (int64_t j = slotq; j < m; j += NSLOTQ) {
      const dv2* p = (const dv2*)(Qi + j * a.mp);
      double t = 0;
#pragma unroll
      for (int r = 0; r < RQ; ++r)
        if (validq[r]) {
          const dv2 v = p[r * GQ + lgq];
          t += v.x * uq[r][0] + v.y * uq[r][1];
        }
      t = gsum<GQ>(t);
      if (lgq == 0) f(j, t);
    }
  };

  // ---- initial state: x = 0, r = rhs, z = Q^{-1} r, d = z
  for (int i = threadIdx.x; i < LV; i += kNT) {
    sx[i] = 0;
    sr[i] = i < m ? a.rhs[i] : 0.0;
    sz[i] = 0;
    sd[i] = 0;
    sq[i] = 0;
  }
  __syncthreads();
  qpass(sr, [&](int64_t j, double t) { sz[j] = t; });
  __syncthreads();
  double rz = 0, rr = 0;
  for (int i = threadIdx.x; i < m; i += kNT) {
    rz += sr[i] * sz[i];
    rr += sr[i] * sr[i];
    sd[i] = sz[i];
  }
  block_sum2(rz, rr, red, lane, wid);
  const double rz0 = rz;
  const double tol2 = a.tol > 0 ? a.tol * a.tol * rz : -1.0;
  int k = 0;
  bool stop = a.max_it <= 0 || !(rz > 0) || rz <= tol2;
  double rz_prev = rz;

  while (!stop) {
    if (k > 0) {  // d_k = z_k + beta_k d_{k-1}
      const double beta = a.inner == SKIPM_INNER_CG ? rz / rz_prev : 0.0;
      for (int i = threadIdx.x; i < m; i += kNT) sd[i] = sz[i] + beta * sd[i];
      __syncthreads();
    }
    // ---- q = A D^2 A^T d: one pass over A
    double uu[R][V], acc[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int row0 = (r * G + lg) * V;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        uu[r][e] = valid[r] ? sd[row0 + e] : 0.0;
        acc[r][e] = 0;
      }
    }
    // columns in chunks of CH per lane group, the next chunk's loads (A and
    // D^2) in flight while this one is used: one memory latency per chunk
    VT cv[CH][R], nv[CH][R];
    double cd2[CH], nd2[CH];
    // loads without branches, so the compiler can keep the next chunk in
    // flight while this one is used: addresses are clamped in bounds, rows
    // past lda are zeroed by a 0/1 factor, and a column past n gets the
    // coefficient 0 (its finite values then add nothing)
    auto load_chunk = [&](VT (*dst)[R], double* dd, int64_t c0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int64_t col = c0 + (int64_t)c * NSLOT;
        const int64_t cc = col < n ? col : n - 1;
        const VT* p = (const VT*)(A + cc * a.lda);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[c][r] = p[vrow[r]] * vmask[r];
        dd[c] = a.d2[cc] * (col < n ? 1.0 : 0.0);
      }
    };
    auto use_chunk = [&](VT (*cvv)[R], const double* dd) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        double t = 0;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) t += (double)cvv[c][r][e] * uu[r][e];
        t = gsum<G>(t);
        const double coef = dd[c] * t;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int e = 0; e < V; ++e) acc[r][e] += coef * (double)cvv[c][r][e];
      }
    };
    // two register buffers used in turn (no copies between them, so the loads
    // of one stay in flight while the other is used)
    const int64_t S = (int64_t)CH * NSLOT;
    int64_t col0 = slot;
    load_chunk(cv, cd2, col0);
    while (col0 < n) {
      if (col0 + S < n) load_chunk(nv, nd2, col0 + S);
      use_chunk(cv, cd2);
      col0 += S;
      if (col0 >= n) break;
      if (col0 + S < n) load_chunk(cv, cd2, col0 + S);
      use_chunk(nv, nd2);
      col0 += S;
    }
    // fold: the groups of a wave, then the waves in order
#pragma unroll
    for (int off = G; off < 64; off <<= 1)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int e = 0; e < V; ++e) acc[r][e] += __shfl_xor(acc[r][e], off, 64);
    if (grp == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int e = 0; e < V; ++e) wbuf[wid * LROWS + (r * G + lg) * V + e] = acc[r][e];
    }
    __syncthreads();
    double dq = 0, unused = 0;
    for (int i = threadIdx.x; i < LV; i += kNT) {
      double s = 0;
      if (i < m && i < LROWS)
        for (int w = 0; w < kNW; ++w) s += wbuf[w * LROWS + i];
      sq[i] = s;
      dq += sd[i] * s;
    }
    block_sum2(dq, unused, red, lane, wid);
    if (!(dq > 0)) break;  // breakdown: the operator lost positive definiteness numerically
    const double alpha = a.inner == SKIPM_INNER_RICHARDSON ? 1.0 : rz / dq;
    // ---- w = Q^{-1} q; x += alpha d, r -= alpha q, z -= alpha w
    qpass(sq, [&](int64_t j, double t) {
      sx[j] += alpha * sd[j];
      sr[j] -= alpha * sq[j];
      sz[j] -= alpha * t;
    });
    __syncthreads();
    double nrz = 0, nrr = 0;
    for (int i = threadIdx.x; i < m; i += kNT) {
      nrz += sr[i] * sz[i];
      nrr += sr[i] * sr[i];
    }
    block_sum2(nrz, nrr, red, lane, wid);
    rz_prev = rz;
    rz = nrz;
    rr = nrr;
    ++k;
    stop = k >= a.max_it || rz <= tol2 || !(rz > 0);
  }
  for (int i = threadIdx.x; i < m; i += kNT) {
    a.x[i] = sx[i];
    if (a.r) a.r[i] = sr[i];
    if (a.z) a.z[i] = sz[i];
    if (a.d) a.d[i] = sd[i];
  }
  if (threadIdx.x == 0) {
    a.sc[S_CG_RZ] = rz;
    a.sc[S_CG_RZ0] = rz0;
    a.sc[S_CG_TOL2] = tol2;
    a.sc[S_V_RR] = rr;
    a.is[I_CG_ITERS] = k;
    a.is[I_CG_MAX] = a.max_it;
    a.is[I_CG_RESID] = 0;
    a.is[I_CG_DONE] = 1;
  }
}

template <typename TA, int G, int R, int GQ, int RQ>
void launch_small(const SmallCg& a, hipStream_t st) {
  hipLaunchKernelGGL((k_cg_small<TA, G, R, GQ, RQ>), dim3(1), dim3(kNT), 0, st, a);
}

}  // namespace

// Shapes follow the lane layouts above: A's leading dimension (a multiple of
// 4) decides G, R; Q^{-1}'s (a multiple of 64) decides GQ, RQ.
int launch_cg_small(const SmallCg& a, int ta, hipStream_t st) {
  if (a.m < 1 || a.m > 128 || a.n < 1 || a.lda < a.m || a.lda % 4 || a.mp < a.m || a.mp % 64 ||
      a.mp > 128)
    return -1;
  // Measured against the multi-workgroup CG (per CG iteration, FP64 A): 8.2
  // against 16.1 us at 40 x 800, 10.5 against 17.8 at 50 x 1000, 16.3
  // against 17.9 at 64 x 2000; with 64-lane column groups (m > 64) and with
  // FP32 copies of A it was slower, so only FP64 A with m <= 64 takes it.
  if (ta != SKIPM_F64 || a.lda > 64) return -1;
  const int qshape = a.mp <= 64 ? 0 : (a.mp <= 128 ? 1 : 2);  // (16,2) (64,1) (64,2)
  if (a.lda <= 32 && qshape == 0) return launch_small<double, 16, 1, 16, 2>(a, st), 0;
  if (a.lda <= 64 && qshape == 0) return launch_small<double, 16, 2, 16, 2>(a, st), 0;
  return -1;
}

}  // namespace skipm
