// Preconditioner build: the Gram matrix Q = B B^T of the sketch B = A D W
// (eq. pdprecond) and its inverse Q^{-1}, applied inside CG as a dense GEMV.
//
// Q^{-1} instead of Q^{-1/2}: CG on the split system of eq. precond_alt and CG
// preconditioned with M = Q on eq. precond produce the same iterates dy
// (Q^{-1/2} z_j = dy_j), so the square root never has to be formed.  The
// inverse is formed as X^T X with X = L^{-1} from a blocked Cholesky factor
// L of Q (two launches per block column), then a blocked triangular inverse
// (one launch per block row) and one launch for X^T X.
#include "common.h"

namespace skipm {

namespace {

// ---------------------------------------------------------------------------
// Gram: Gpart[ks] = B[:, cols of split ks] B[:, same]^T, 128 x 128 tiles of the
// lower triangle, mirrored to the upper triangle.  G is mp x mp, column-major.
//
// On the FP64 matrix cores: v_mfma_f64_16x16x4 takes, in lane l, A[l%16][l/16]
// of a 16x4 block and B[l/16][l%16] of a 4x16 block, and accumulates
// D[l/16 + 4r][l%16] in element r of the lane's four-double accumulator.  The
// four waves of a workgroup own a 64 x 64 quarter of the tile each (4 x 4
// blocks of 16 x 16).  Per stage of 16 columns of B, the tile's two 128-row
// panels go through LDS (two buffers: the next stage's loads are in flight in
// registers while this stage's 64 MFMAs per wave run; one barrier per stage).
// Every entry is a sum over the split's columns in increasing order.
// ---------------------------------------------------------------------------
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef double dacc4 __attribute__((ext_vector_type(4)));
constexpr int kRT = 128;      // output tile
constexpr int kRK = 16;       // columns of B per stage
constexpr int kRP = kRT + 2;  // LDS row pitch (16-byte aligned rows)

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ B, int64_t ldb,
                                              int64_t m, int64_t w, double* __restrict__ Gpart,
                                              int64_t mp, int64_t cols_per_split) {
  __shared__ double Ai[2][kRK][kRP];
  __shared__ double Aj[2][kRK][kRP];
  // decode the lower-triangle tile pair (ti >= tj)
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int ks = blockIdx.y;
  const int64_t i0 = (int64_t)ti * kRT, j0 = (int64_t)tj * kRT;
  const int64_t cb = (int64_t)ks * cols_per_split;
  const int64_t ce = cb + cols_per_split < w ? cb + cols_per_split : w;
  const int th = threadIdx.x, lane = th & 63, wv = th >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  // load mapping: 4 x (one column kk of the stage, rows 2 rp and 2 rp + 1) per panel
  const int a_kk = th >> 6, a_rp = th & 63;
  dvec2 ri[4], rj[4];
  auto pair = [&](const int64_t r, const int64_t c) {
    dvec2 v = (dvec2)0.0;
    if (c < ce) {
      const double* p = B + c * ldb + r;
      if (r + 1 < m) {
        v = *(const dvec2*)p;
      } else if (r < m) {
        v.x = p[0];
      }
    }
    return v;
  };
  auto fetch = [&](const int64_t c0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t c = c0 + a_kk + 4 * q;
      ri[q] = pair(i0 + 2 * a_rp, c);
      rj[q] = pair(j0 + 2 * a_rp, c);
    }
  };
  auto stash = [&](const int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *(dvec2*)&Ai[b][a_kk + 4 * q][2 * a_rp] = ri[q];
      *(dvec2*)&Aj[b][a_kk + 4 * q][2 * a_rp] = rj[q];
    }
  };
  dacc4 acc[4][4];
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = (dacc4)0.0;
  const int64_t nst = ce > cb ? (ce - cb + kRK - 1) / kRK : 0;
  if (nst > 0) {
    fetch(cb);
    stash(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int b = (int)(st & 1);
    if (st + 1 < nst) fetch(cb + (st + 1) * kRK);
#pragma unroll
    for (int s4 = 0; s4 < kRK / 4; ++s4) {
      double fa[4], fb[4];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) fa[ib] = Ai[b][4 * s4 + lk][64 * wr + 16 * ib + li];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) fb[jb] = Aj[b][4 * s4 + lk][64 * wc + 16 * jb + li];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[ib], fb[jb], acc[ib][jb], 0, 0, 0);
    }
    if (st + 1 < nst) stash(b ^ 1);
    __syncthreads();
  }
  // element (i, k) of the tile, mirrored; on a diagonal tile only i >= k is
  // written (with its mirror), so every entry has exactly one writer
  double* G = Gpart + (int64_t)ks * mp * mp;
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 64 * wr + 16 * ib + lk + 4 * r;
        const int64_t k = j0 + 64 * wc + 16 * jb + li;
        if (i < mp && k < mp && (ti != tj || i >= k)) {
          G[i + k * mp] = acc[ib][jb][r];
          G[k + i * mp] = acc[ib][jb][r];
        }
      }
}

// G = sum of the split partials on the m x m block; identity on the padding.
__global__ __launch_bounds__(256) void k_gram_finish(const double* __restrict__ Gpart, int ksplit,
                                                     int64_t m, int64_t mp,
                                                     double* __restrict__ G) {
  const int64_t total = mp * mp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % mp, k = e / mp;
    double v;
    if (i < m && k < m) {
      v = 0;
      for (int q = 0; q < ksplit; ++q) v += Gpart[(int64_t)q * total + e];
    } else {
      v = (i == k) ? 1.0 : 0.0;
    }
    G[e] = v;
  }
}

__global__ __launch_bounds__(256) void k_shift_diag(double* __restrict__ G, int64_t mp, int64_t m,
                                                    double rel) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) G[i + i * mp] *= (1.0 + rel);
}

// ---------------------------------------------------------------------------
// Blocked Cholesky G = L L^T (lower, in place), explicit X = L^{-1} (block lower
// triangular, stored in Xb) and P = X^T X = G^{-1} (written over G).
// P is applied by one GEMV per CG iteration.  Because L is a backward-stable
// factor and X has a small residual, X^T X G has eigenvalues within u*kappa(G)
// of one, unlike a Gauss-Jordan inverse of G.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Panel step k, one wave of NB lanes per block.  Every block factors G_kk with
// lane i holding row i in registers (left-looking: column p needs row p's
// finished entries, taken from lane p by readlane), then keeps L_kk in LDS.
// Block 0 forms X_kk = L_kk^{-1} (lane c solves column c by forward
// substitution, reading L_kk by LDS broadcast) and stores it in Xb; block
// b > 0 solves L_kk y = G_ik[r, :]^T for its rows r (lane r), i.e.
// L_ik = G_ik L_kk^{-T}, in place.
template <int NB>
__global__ __launch_bounds__(NB) void k_chol_panel(double* __restrict__ G, double* __restrict__ Xb,
                                                   int64_t mp, int k,
                                                   int32_t* __restrict__ fail) {
  __shared__ double Ls[NB][NB + 1];
  __shared__ double rdiag[NB];
  const int lane = threadIdx.x;
  const int64_t K0 = (int64_t)k * NB;
  double a[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) a[j] = G[(K0 + lane) + (K0 + j) * mp];
  bool bad = false;
#pragma unroll
  for (int p = 0; p < NB; ++p) {
    double s = a[p];
#pragma unroll
    for (int q = 0; q < p; ++q) s -= a[q] * readlane_d(a[q], p);
    double d = readlane_d(s, p);
    if (!(d > 0.0)) {
      bad = true;
      d = 1e-300;
    }
    const double lpp = sqrt(d);
    a[p] = lane > p ? s / lpp : (lane == p ? lpp : 0.0);
  }
  if (bad && lane == 0) atomicOr(fail, 1);
#pragma unroll
  for (int j = 0; j < NB; ++j) Ls[lane][j] = a[j];
  __syncthreads();
  rdiag[lane] = 1.0 / Ls[lane][lane];
  __syncthreads();
  if (blockIdx.x == 0) {
    // column `lane` of L_kk^{-1}
    double x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < i; ++q) s -= Ls[i][q] * x[q];
      x[i] = s * rdiag[i];
    }
    __syncthreads();
    // stage through LDS (transpose) for coalesced stores of the column-major tile
#pragma unroll
    for (int i = 0; i < NB; ++i) Ls[i][lane] = x[i];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NB; ++c) Xb[(K0 + lane) + (K0 + c) * mp] = Ls[lane][c];
    return;
  }
  const int64_t I0 = K0 + (int64_t)blockIdx.x * NB;
  double y[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) y[c] = G[(I0 + lane) + (K0 + c) * mp];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    double s = y[c];
#pragma unroll
    for (int q = 0; q < c; ++q) s -= Ls[c][q] * y[q];
    y[c] = s * rdiag[c];
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) G[(I0 + lane) + (K0 + c) * mp] = y[c];
}

// C[I, J] (+)= sign * sum_q A[I, q-block] B[J, q-block]^T over a range of q
// blocks, with NB x NB tiles staged through LDS (16 x 16 threads, TW x TW each).
template <int NB>
struct TileAcc {
  static constexpr int TW = NB / 16;
  double acc[TW][TW];
  __device__ void zero() {
#pragma unroll
    for (int p = 0; p < TW; ++p)
#pragma unroll
      for (int o = 0; o < TW; ++o) acc[p][o] = 0.0;
  }
  // acc += At * Bt^T   (At, Bt: NB x NB tiles in LDS, row index first)
  __device__ void mma_nt(double (*At)[NB + 1], double (*Bt)[NB + 1]) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int q = 0; q < NB; ++q) {
      double a[TW], b[TW];
#pragma unroll
      for (int p = 0; p < TW; ++p) {
        a[p] = At[ty * TW + p][q];
        b[p] = Bt[tx * TW + p][q];
      }
#pragma unroll
      for (int p = 0; p < TW; ++p)
#pragma unroll
        for (int o = 0; o < TW; ++o) acc[p][o] += a[p] * b[o];
    }
  }
  // acc += At^T * Bt
  __device__ void mma_tn(double (*At)[NB + 1], double (*Bt)[NB + 1]) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int q = 0; q < NB; ++q) {
      double a[TW], b[TW];
#pragma unroll
      for (int p = 0; p < TW; ++p) {
        a[p] = At[q][ty * TW + p];
        b[p] = Bt[q][tx * TW + p];
      }
#pragma unroll
      for (int p = 0; p < TW; ++p)
#pragma unroll
        for (int o = 0; o < TW; ++o) acc[p][o] += a[p] * b[o];
    }
  }
  // acc += At * Bt
  __device__ void mma_nn(double (*At)[NB + 1], double (*Bt)[NB + 1]) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int q = 0; q < NB; ++q) {
      double a[TW], b[TW];
#pragma unroll
      for (int p = 0; p < TW; ++p) {
        a[p] = At[ty * TW + p][q];
        b[p] = Bt[q][tx * TW + p];
      }
#pragma unroll
      for (int p = 0; p < TW; ++p)
#pragma unroll
        for (int o = 0; o < TW; ++o) acc[p][o] += a[p] * b[o];
    }
  }
};

template <int NB>
__device__ void load_tile(double (*Tt)[NB + 1], const double* __restrict__ M, int64_t ld,
                          int64_t r0, int64_t c0) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int r = e % NB, c = e / NB;
    Tt[r][c] = M[(r0 + r) + (c0 + c) * ld];
  }
}

// Trailing update of step k: G_ij -= L_ik L_jk^T for k < j <= i (lower triangle).
template <int NB>
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ G, int64_t mp, int k) {
  __shared__ double Ai[NB][NB + 1];
  __shared__ double Aj[NB][NB + 1];
  int t = blockIdx.x, di = 0;  // decode (di >= dj) over the trailing blocks
  while (t > di) {
    t -= di + 1;
    ++di;
  }
  const int bi = k + 1 + di, bj = k + 1 + t;
  const int64_t K0 = (int64_t)k * NB, I0 = (int64_t)bi * NB, J0 = (int64_t)bj * NB;
  load_tile<NB>(Ai, G, mp, I0, K0);
  load_tile<NB>(Aj, G, mp, J0, K0);
  __syncthreads();
  TileAcc<NB> ta;
  ta.zero();
  ta.mma_nt(Ai, Aj);
  constexpr int TW = NB / 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int p = 0; p < TW; ++p)
#pragma unroll
    for (int o = 0; o < TW; ++o) {
      const int64_t gi = I0 + ty * TW + p, gj = J0 + tx * TW + o;
      G[gi + gj * mp] -= ta.acc[p][o];
    }
}

// X = L^{-1} from its diagonal blocks by recursive doubling.  At a level with
// ranges of `half` blocks, pair p joins a = [a0, a0 + half) and the range b that
// follows it (at most `half` blocks); with X_aa and X_bb already inverses,
//   X_ba = -X_bb (L_ba X_aa).
// k_trinv_c forms C = L_ba X_aa (X_aa lower triangular: tile (i, c) needs
// blocks j >= c), k_trinv_x then X_ba = -X_bb C (tile (r, c) needs j <= r).
// Grid: (half, half, pairs), one workgroup per tile.
template <int NB>
__global__ __launch_bounds__(256) void k_trinv_c(const double* __restrict__ G,
                                                 const double* __restrict__ Xb,
                                                 double* __restrict__ Ct, int64_t mp, int half,
                                                 int T) {
  __shared__ double At[NB][NB + 1];
  __shared__ double Bt[NB][NB + 1];
  const int a0 = blockIdx.z * 2 * half, b0 = a0 + half;
  const int nbb = T - b0 < half ? T - b0 : half;
  const int ai = blockIdx.x, bi = blockIdx.y;
  if (bi >= nbb) return;
  const int64_t R0 = (int64_t)(b0 + bi) * NB, C0 = (int64_t)(a0 + ai) * NB;
  TileAcc<NB> ta;
  ta.zero();
  for (int j = ai; j < half; ++j) {
    const int64_t J0 = (int64_t)(a0 + j) * NB;
    __syncthreads();
    load_tile<NB>(At, G, mp, R0, J0);   // L_(b0+bi),(a0+j)
    load_tile<NB>(Bt, Xb, mp, J0, C0);  // X_(a0+j),(a0+ai)
    __syncthreads();
    ta.mma_nn(At, Bt);
  }
  constexpr int TW = NB / 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int p = 0; p < TW; ++p)
#pragma unroll
    for (int o = 0; o < TW; ++o)
      Ct[(R0 + ty * TW + p) + (C0 + tx * TW + o) * mp] = ta.acc[p][o];
}

template <int NB>
__global__ __launch_bounds__(256) void k_trinv_x(const double* __restrict__ Ct,
                                                 double* __restrict__ Xb, int64_t mp, int half,
                                                 int T) {
  __shared__ double At[NB][NB + 1];
  __shared__ double Bt[NB][NB + 1];
  const int a0 = blockIdx.z * 2 * half, b0 = a0 + half;
  const int nbb = T - b0 < half ? T - b0 : half;
  const int ai = blockIdx.x, bi = blockIdx.y;
  if (bi >= nbb) return;
  const int64_t R0 = (int64_t)(b0 + bi) * NB, C0 = (int64_t)(a0 + ai) * NB;
  TileAcc<NB> ta;
  ta.zero();
  for (int j = 0; j <= bi; ++j) {
    const int64_t J0 = (int64_t)(b0 + j) * NB;
    __syncthreads();
    load_tile<NB>(At, Xb, mp, R0, J0);  // X_(b0+bi),(b0+j)
    load_tile<NB>(Bt, Ct, mp, J0, C0);  // C_(b0+j),(a0+ai)
    __syncthreads();
    ta.mma_nn(At, Bt);
  }
  constexpr int TW = NB / 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int p = 0; p < TW; ++p)
#pragma unroll
    for (int o = 0; o < TW; ++o)
      Xb[(R0 + ty * TW + p) + (C0 + tx * TW + o) * mp] = -ta.acc[p][o];
}

// P = X^T X: P_ij = sum_{l >= i} X_li^T X_lj for j <= i, mirrored; written over G.
template <int NB>
__global__ __launch_bounds__(256) void k_xtx(const double* __restrict__ Xb, double* __restrict__ G,
                                             int64_t mp, int T) {
  __shared__ double At[NB][NB + 1];
  __shared__ double Bt[NB][NB + 1];
  int t = blockIdx.x, bi = 0;
  while (t > bi) {
    t -= bi + 1;
    ++bi;
  }
  const int bj = t;
  const int64_t I0 = (int64_t)bi * NB, J0 = (int64_t)bj * NB;
  TileAcc<NB> ta;
  ta.zero();
  for (int l = bi; l < T; ++l) {
    const int64_t L0 = (int64_t)l * NB;
    __syncthreads();
    load_tile<NB>(At, Xb, mp, L0, I0);  // X_li
    load_tile<NB>(Bt, Xb, mp, L0, J0);  // X_lj
    __syncthreads();
    ta.mma_tn(At, Bt);
  }
  constexpr int TW = NB / 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int p = 0; p < TW; ++p)
#pragma unroll
    for (int o = 0; o < TW; ++o) {
      const int64_t gi = I0 + ty * TW + p, gj = J0 + tx * TW + o;
      G[gi + gj * mp] = ta.acc[p][o];
      G[gj + gi * mp] = ta.acc[p][o];
    }
}

// Out = X * In for X block-lower-triangular (mp x mp, ld mp; only blocks
// k <= i are read) and In with nrows valid rows (ld ldin; rows beyond are zero)
// and ncols columns.  Rows < nrows_out of Out are written.
template <int NB>
__global__ __launch_bounds__(256) void k_trmm(const double* __restrict__ X, int64_t mp,
                                              const double* __restrict__ In, int64_t ldin,
                                              int64_t nrows, int64_t ncols,
                                              double* __restrict__ Out, int64_t ldout,
                                              int64_t nrows_out) {
  __shared__ double At[NB][NB + 1];
  __shared__ double Bt[NB][NB + 1];
  const int bi = blockIdx.x;
  const int64_t I0 = (int64_t)bi * NB, J0 = (int64_t)blockIdx.y * NB;
  TileAcc<NB> ta;
  ta.zero();
  for (int kb = 0; kb <= bi; ++kb) {
    const int64_t K0 = (int64_t)kb * NB;
    __syncthreads();
    load_tile<NB>(At, X, mp, I0, K0);
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
      const int r = e % NB, c = e / NB;
      const int64_t gr = K0 + r, gc = J0 + c;
      Bt[r][c] = (gr < nrows && gc < ncols) ? In[gr + gc * ldin] : 0.0;
    }
    __syncthreads();
    ta.mma_nn(At, Bt);
  }
  constexpr int TW = NB / 16;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int p = 0; p < TW; ++p)
#pragma unroll
    for (int o = 0; o < TW; ++o) {
      const int64_t gi = I0 + ty * TW + p, gj = J0 + tx * TW + o;
      if (gi < nrows_out && gj < ncols) Out[gi + gj * ldout] = ta.acc[p][o];
    }
}

// G_ii += c * trace(G) for i < m (single workgroup): the shift of shifted
// Cholesky QR, with ||B||_2^2 bounded by ||B||_F^2 = trace(B B^T).
__global__ __launch_bounds__(1024) void k_shift_trace(double* __restrict__ G, int64_t mp, int64_t m,
                                                      double c) {
  __shared__ double buf[16];
  double tr = 0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) tr += G[i + i * mp];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
  if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = tr;
  __syncthreads();
  double tot = 0;
  for (int q = 0; q < 16; ++q) tot += buf[q];
  for (int64_t i = threadIdx.x; i < m; i += 1024) G[i + i * mp] += c * tot;
}

}  // namespace

// Splits of the Gram along the columns of B: at most 16, slices of at least
// 64 columns, at most 64 MiB of partials; among those, the count with the
// least estimated time, in columns of one workgroup: rounds of 256
// workgroups (one per CU: a CU that runs two runs each at about half rate)
// times the columns per split, plus the finish's read of the partials
// (about 8 columns' time per 1024 x 1024 partial).  At m = 1000 (36 tiles),
// 7 splits in one round take 110 us where 8 (288 workgroups) took 146.
int gram_ksplit(int64_t mp, int64_t w) {
  const int64_t T = (mp + kRT - 1) / kRT, ntiles = T * (T + 1) / 2;
  int64_t kmax = std::min<int64_t>(16, w / 64);
  kmax = std::min<int64_t>(kmax, (int64_t)(64ll << 20) / (8 * mp * mp));
  int64_t best = 1;
  double best_cost = HUGE_VAL;
  for (int64_t ks = 1; ks <= kmax; ++ks) {
    const int64_t cps = ((w + ks - 1) / ks + 15) / 16 * 16;
    const int64_t rounds = (ntiles * ks + 255) / 256;
    const double cost = (double)(rounds * cps) + (double)ks * (double)(mp * mp) / 131072.0;
    if (cost < best_cost) {
      best_cost = cost;
      best = ks;
    }
  }
  return (int)best;
}

void launch_gram(const double* B, int64_t ldb, int64_t m, int64_t w, double* Gpart, int ksplit,
                 int64_t mp, hipStream_t st) {
  const int T = (int)((mp + kRT - 1) / kRT);
  const int ntiles = T * (T + 1) / 2;
  int64_t cps = (w + ksplit - 1) / ksplit;
  cps = (cps + 15) / 16 * 16;
  hipLaunchKernelGGL(k_gram, dim3(ntiles, ksplit), dim3(256), 0, st, B, ldb, m, w, Gpart, mp,
                     cps);
}

void launch_gram_finish(const double* Gpart, int ksplit, int64_t m, int64_t mp, double* G,
                        hipStream_t st) {
  int64_t blocks = (mp * mp + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)blocks), dim3(256), 0, st, Gpart, ksplit, m,
                     mp, G);
}

// Cholesky block (panel width) of every factorisation: mp is a multiple of 64,
// so of 32; 32 x 32 FP64 tiles keep a panel's rows in one wave's registers.
constexpr int kNb = 32;

void launch_spd_inverse(double* G, double* Xb, double* Ct, int64_t mp, int32_t* fail,
                        hipStream_t st) {
  const int T = (int)(mp / kNb);
  for (int k = 0; k < T; ++k) {
    const int rest = T - k - 1;
    hipLaunchKernelGGL(k_chol_panel<kNb>, dim3(rest + 1), dim3(kNb), 0, st, G, Xb, mp, k, fail);
    if (rest > 0)
      hipLaunchKernelGGL(k_chol_update<kNb>, dim3(rest * (rest + 1) / 2), dim3(256), 0, st, G,
                         mp, k);
  }
  // X = L^{-1}: log2(T) levels of two launches each
  for (int half = 1; half < T; half *= 2) {
    const dim3 grid(half, half, (T + 2 * half - 1) / (2 * half));
    hipLaunchKernelGGL(k_trinv_c<kNb>, grid, dim3(256), 0, st, G, Xb, Ct, mp, half, T);
    hipLaunchKernelGGL(k_trinv_x<kNb>, grid, dim3(256), 0, st, Ct, Xb, mp, half, T);
  }
  const int npairs = T * (T + 1) / 2;
  hipLaunchKernelGGL(k_xtx<kNb>, dim3(npairs), dim3(256), 0, st, Xb, G, mp, T);
}

void launch_shift_diag(double* G, int64_t mp, int64_t m, double rel, hipStream_t st) {
  hipLaunchKernelGGL(k_shift_diag, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, G, mp, m,
                     rel);
}

void launch_trmm(const double* X, int64_t mp, const double* In, int64_t ldin, int64_t nrows,
                 int64_t ncols, double* Out, int64_t ldout, int64_t nrows_out, hipStream_t st) {
  const int T = (int)(mp / kNb);
  const unsigned gy = (unsigned)((ncols + kNb - 1) / kNb);
  hipLaunchKernelGGL(k_trmm<kNb>, dim3(T, gy), dim3(256), 0, st, X, mp, In, ldin, nrows, ncols,
                     Out, ldout, nrows_out);
}

void launch_shift_trace(double* G, int64_t mp, int64_t m, double c, hipStream_t st) {
  hipLaunchKernelGGL(k_shift_trace, dim3(1), dim3(1024), 0, st, G, mp, m, c);
}

}  // namespace skipm
