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
// Gram: Gpart[ks] = B[:, cols of split ks] B[:, same]^T, RT x RT tiles of the
// lower triangle (RT = 128, or 64 when mp <= 256), mirrored to the upper
// triangle.  G is mp x mp, column-major.
//
// On the FP64 matrix cores: v_mfma_f64_16x16x4 takes, in lane l, A[l%16][l/16]
// of a 16x4 block and B[l/16][l%16] of a 4x16 block, and accumulates
// D[l/16 + 4r][l%16] in element r of the lane's four-double accumulator.  The
// four waves of a workgroup own an RT/2 x RT/2 quarter of the tile each
// (RT/32 x RT/32 blocks of 16 x 16).  Per stage of 16 columns of B, the tile's
// two RT-row panels go through LDS (two buffers: the next stage's loads are in
// flight in registers while this stage's MFMAs run; one barrier per stage).
// Every entry is a sum over the split's columns in increasing order, in the
// same steps for either tile size.
// ---------------------------------------------------------------------------
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef double dacc4 __attribute__((ext_vector_type(4)));
constexpr int kRT = 128;      // output tile of the split rule
constexpr int kRK = 16;       // columns of B per stage

template <int RT>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ B, int64_t ldb,
                                              int64_t m, int64_t w, double* __restrict__ Gpart,
                                              int64_t mp, int64_t cols_per_split) {
  constexpr int RP = RT + 2;       // LDS row pitch (16-byte aligned rows)
  constexpr int NBW = RT / 32;     // 16 x 16 blocks per wave and dimension
  constexpr int TPC = RT / 2;      // threads per panel column (two rows each)
  constexpr int CPP = 256 / TPC;   // panel columns per pass of the workgroup
  constexpr int NPASS = kRK / CPP;
  __shared__ double Ai[2][kRK][RP];
  __shared__ double Aj[2][kRK][RP];
  // decode the lower-triangle tile pair (ti >= tj)
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int ks = blockIdx.y;
  const int64_t i0 = (int64_t)ti * RT, j0 = (int64_t)tj * RT;
  const int64_t cb = (int64_t)ks * cols_per_split;
  const int64_t ce = cb + cols_per_split < w ? cb + cols_per_split : w;
  const int th = threadIdx.x, lane = th & 63, wv = th >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  // load mapping: NPASS x (one column kk of the stage, rows 2 rp and 2 rp + 1) per panel
  const int a_kk = th / TPC, a_rp = th % TPC;
  dvec2 ri[NPASS], rj[NPASS];
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
    for (int q = 0; q < NPASS; ++q) {
      const int64_t c = c0 + a_kk + CPP * q;
      ri[q] = pair(i0 + 2 * a_rp, c);
      rj[q] = pair(j0 + 2 * a_rp, c);
    }
  };
  auto stash = [&](const int b) {
#pragma unroll
    for (int q = 0; q < NPASS; ++q) {
      *(dvec2*)&Ai[b][a_kk + CPP * q][2 * a_rp] = ri[q];
      *(dvec2*)&Aj[b][a_kk + CPP * q][2 * a_rp] = rj[q];
    }
  };
  dacc4 acc[NBW][NBW];
#pragma unroll
  for (int ib = 0; ib < NBW; ++ib)
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb) acc[ib][jb] = (dacc4)0.0;
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
      double fa[NBW], fb[NBW];
#pragma unroll
      for (int ib = 0; ib < NBW; ++ib) fa[ib] = Ai[b][4 * s4 + lk][(RT / 2) * wr + 16 * ib + li];
#pragma unroll
      for (int jb = 0; jb < NBW; ++jb) fb[jb] = Aj[b][4 * s4 + lk][(RT / 2) * wc + 16 * jb + li];
#pragma unroll
      for (int ib = 0; ib < NBW; ++ib)
#pragma unroll
        for (int jb = 0; jb < NBW; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[ib], fb[jb], acc[ib][jb], 0, 0, 0);
    }
    if (st + 1 < nst) stash(b ^ 1);
    __syncthreads();
  }
  // element (i, k) of the tile, mirrored; on a diagonal tile only i >= k is
  // written (with its mirror), so every entry has exactly one writer
  double* G = Gpart + (int64_t)ks * mp * mp;
#pragma unroll
  for (int ib = 0; ib < NBW; ++ib)
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + (RT / 2) * wr + 16 * ib + lk + 4 * r;
        const int64_t k = j0 + (RT / 2) * wc + 16 * jb + li;
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

// One NB x NB output tile (NB = 32) of a product of tiles staged through LDS,
// on the FP64 matrix cores: wave w of the workgroup's four owns the 16 x 16
// quadrant (w >> 1, w & 1) and takes one v_mfma_f64_16x16x4 per four values
// of the inner index q (in lane l: A[l%16][l/16] of the 16 x 4 block,
// B[l/16][l%16] of the 4 x 16 block; D[l/16 + 4r][l%16] in element r of the
// accumulator).  Every entry is a sum over q in increasing order.
template <int NB>
struct TileAcc {
  static_assert(NB == 32, "four waves of 16 x 16 quadrants");
  dacc4 acc;
  int i0, j0, li, lk;
  __device__ TileAcc() {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    i0 = 16 * (w >> 1);
    j0 = 16 * (w & 1);
    li = lane & 15;
    lk = lane >> 4;
    acc = (dacc4)0.0;
  }
  __device__ void zero() { acc = (dacc4)0.0; }
  // acc += At * Bt^T   (At, Bt: NB x NB tiles in LDS, row index first)
  __device__ void mma_nt(double (*At)[NB + 1], double (*Bt)[NB + 1]) {
#pragma unroll
    for (int q0 = 0; q0 < NB; q0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(At[i0 + li][q0 + lk], Bt[j0 + li][q0 + lk], acc,
                                                 0, 0, 0);
  }
  // acc += At^T * Bt
  __device__ void mma_tn(double (*At)[NB + 1], double (*Bt)[NB + 1]) {
#pragma unroll
    for (int q0 = 0; q0 < NB; q0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(At[q0 + lk][i0 + li], Bt[q0 + lk][j0 + li], acc,
                                                 0, 0, 0);
  }
  // acc += At * Bt
  __device__ void mma_nn(double (*At)[NB + 1], double (*Bt)[NB + 1]) {
#pragma unroll
    for (int q0 = 0; q0 < NB; q0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(At[i0 + li][q0 + lk], Bt[q0 + lk][j0 + li], acc,
                                                 0, 0, 0);
  }
  // the tile row and column of element r of the accumulator
  __device__ int row(int r) const { return i0 + lk + 4 * r; }
  __device__ int col() const { return j0 + li; }
};

template <int NB>
__device__ void load_tile(double (*Tt)[NB + 1], const double* __restrict__ M, int64_t ld,
                          int64_t r0, int64_t c0) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int r = e % NB, c = e / NB;
    Tt[r][c] = M[(r0 + r) + (c0 + c) * ld];
  }
}

// One NB x NB tile in the registers of a 256-thread workgroup (element
// threadIdx.x + 256 q at row e % NB, column e / NB, as load_tile), so that
// the loops over tile products below request kTileAhead tiles' loads at once
// and wait for their latency once per batch instead of once per tile.
constexpr int kTileAhead = 8;
template <int NB>
struct TileRegs {
  static constexpr int NE = NB * NB / 256;
  double v[NE];
  __device__ void load(const double* __restrict__ M, int64_t ld, int64_t r0, int64_t c0) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + 256 * q;
      v[q] = M[(r0 + e % NB) + (c0 + e / NB) * ld];
    }
  }
  // rows >= nrows or columns >= ncols of M read as zero
  __device__ void load_masked(const double* __restrict__ M, int64_t ld, int64_t r0, int64_t c0,
                              int64_t nrows, int64_t ncols) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int64_t gr = r0 + e % NB, gc = c0 + e / NB;
      v[q] = (gr < nrows && gc < ncols) ? M[gr + gc * ld] : 0.0;
    }
  }
  __device__ void store(double (*Tt)[NB + 1]) const {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + 256 * q;
      Tt[e % NB][e / NB] = v[q];
    }
  }
};

// Trailing update of step kp on tile (bi, bj), bi >= bj > kp:
// G_ij -= L_i,kp L_j,kp^T (all 256 threads of the workgroup).
template <int NB>
__device__ __forceinline__ void update_tile(double* __restrict__ G, int64_t mp, int kp, int bi,
                                            int bj, double (*Ai)[NB + 1], double (*Aj)[NB + 1]) {
  const int64_t P0 = (int64_t)kp * NB, I0 = (int64_t)bi * NB, J0 = (int64_t)bj * NB;
  load_tile<NB>(Ai, G, mp, I0, P0);
  load_tile<NB>(Aj, G, mp, J0, P0);
  __syncthreads();
  TileAcc<NB> ta;
  ta.mma_nt(Ai, Aj);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t gi = I0 + ta.row(r), gj = J0 + ta.col();
    G[gi + gj * mp] -= ta.acc[r];
  }
}

// Step k of the blocked factorisation, one launch of 256-thread workgroups.
// Workgroups 0..rest (rest = T - k - 1) are the panel of column block k: each
// first applies step k-1's update to the diagonal block and to its own block
// of the column (the same sums, in the same order, as the tile update below),
// then wave 0 factors G_kk with lane i holding row i in registers
// (left-looking: column p needs row p's finished entries, taken from lane p by
// readlane).  Workgroup 0 forms X_kk = L_kk^{-1} (lane c solves column c by
// forward substitution, reading L_kk by LDS broadcast) and stores it in Xb;
// workgroup b > 0 solves L_kk y = G_ik[r, :]^T for its rows r (lane r), i.e.
// L_ik = G_ik L_kk^{-T}, in place.  The workgroups after those apply step
// k-1's update to the trailing tiles right of column block k, so the panel
// and the rest of the previous step's update share one launch.
template <int NB>
__global__ __launch_bounds__(256) void k_chol_step(double* __restrict__ G, double* __restrict__ Xb,
                                                   int64_t mp, int k, int T,
                                                   int32_t* __restrict__ fail) {
  static_assert(NB == 32, "the panel keeps a 32 x 32 block in one wave's registers");
  __shared__ double Ai[NB][NB + 1];
  __shared__ double Aj[NB][NB + 1];
  __shared__ double Dg[NB][NB + 1];
  __shared__ double Yb[NB][NB + 1];
  __shared__ double rdiag[NB];
  const int rest = T - k - 1;
  if ((int)blockIdx.x > rest) {  // trailing tile (di >= dj) of step k-1's update
    int t = (int)blockIdx.x - rest - 1, di = 0;
    while (t > di) {
      t -= di + 1;
      ++di;
    }
    update_tile<NB>(G, mp, k - 1, k + 1 + di, k + 1 + t, Ai, Aj);
    return;
  }
  const int bid = blockIdx.x;
  const int64_t K0 = (int64_t)k * NB;
  const int64_t I0 = K0 + (int64_t)bid * NB;  // block b > 0: its rows of column block k
  load_tile<NB>(Dg, G, mp, K0, K0);
  if (bid > 0) load_tile<NB>(Yb, G, mp, I0, K0);
  if (k > 0) {
    load_tile<NB>(Aj, G, mp, K0, K0 - NB);
    if (bid > 0) load_tile<NB>(Ai, G, mp, I0, K0 - NB);
  }
  __syncthreads();
  if (k > 0) {
    TileAcc<NB> td, tb;
    td.mma_nt(Aj, Aj);
    if (bid > 0) tb.mma_nt(Ai, Aj);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Dg[td.row(r)][td.col()] -= td.acc[r];
      if (bid > 0) Yb[tb.row(r)][tb.col()] -= tb.acc[r];
    }
    __syncthreads();
  }
  // wave 0 factors G_kk; its lanes past NB repeat lane NB - 1 and store nothing
  const int lane = threadIdx.x;
  const int ln = lane < NB ? lane : NB - 1;
  if (threadIdx.x < 64) {
    double a[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) a[j] = Dg[ln][j];
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
      a[p] = ln > p ? s / lpp : (ln == p ? lpp : 0.0);
    }
    if (bad && lane == 0) atomicOr(fail, 1);
    // L_kk over the diagonal block (every lane has read its row)
    if (lane < NB) {
#pragma unroll
      for (int j = 0; j < NB; ++j) Dg[lane][j] = a[j];
    }
  }
  __syncthreads();
  if (lane < NB) rdiag[lane] = 1.0 / Dg[lane][lane];
  __syncthreads();
  if (bid == 0) {
    // column `lane` of L_kk^{-1}
    double x[NB];
    if (lane < NB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) s -= Dg[i][q] * x[q];
        x[i] = s * rdiag[i];
      }
      // stage through LDS (transpose) for coalesced stores of the column-major tile
#pragma unroll
      for (int i = 0; i < NB; ++i) Ai[i][lane] = x[i];
    }
    __syncthreads();
    if (lane < NB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) Xb[(K0 + lane) + (K0 + c) * mp] = Ai[lane][c];
    }
    return;
  }
  if (lane < NB) {
    double y[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) y[c] = Yb[lane][c];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double s = y[c];
#pragma unroll
      for (int q = 0; q < c; ++q) s -= Dg[c][q] * y[q];
      y[c] = s * rdiag[c];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) G[(I0 + lane) + (K0 + c) * mp] = y[c];
  }
}

// The whole inverse at mp = 64 (two 32-column blocks) in one workgroup: the
// same steps, sums and orders as the launches for any mp (k_chol_step for
// k = 0 and 1, one level of k_trinv_c / k_trinv_x, k_xtx), with the blocks in
// LDS between them, so a small LP's factorization is one launch instead of
// five.  Wave 0 factors the diagonal blocks; the diagonal block's inverse and
// the solve for the rows below run on waves 0 and 1 side by side.
__device__ __forceinline__ void chol_factor_block(double (*Dg)[33], double* rdiag,
                                                  int32_t* __restrict__ fail) {
  constexpr int NB = 32;
  const int lane = threadIdx.x;
  const int ln = lane < NB ? lane : NB - 1;
  if (threadIdx.x < 64) {
    double a[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) a[j] = Dg[ln][j];
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
      a[p] = ln > p ? s / lpp : (ln == p ? lpp : 0.0);
    }
    if (bad && lane == 0) atomicOr(fail, 1);
    if (lane < NB) {
#pragma unroll
      for (int j = 0; j < NB; ++j) Dg[lane][j] = a[j];
    }
  }
  __syncthreads();
  if (lane < NB) rdiag[lane] = 1.0 / Dg[lane][lane];
  __syncthreads();
}

// column c of L^{-1} (lane c < 32 of its wave), into X[i][c]
__device__ __forceinline__ void chol_inverse_block(double (*Dg)[33], const double* rdiag,
                                                   double (*X)[33], int c) {
  constexpr int NB = 32;
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < i; ++q) s -= Dg[i][q] * x[q];
    x[i] = s * rdiag[i];
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) X[i][c] = x[i];
}

// row r of Y L^{-T} (lane r < 32 of its wave), in place
__device__ __forceinline__ void chol_solve_row(double (*Dg)[33], const double* rdiag,
                                               double (*Y)[33], int r) {
  constexpr int NB = 32;
  double y[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) y[c] = Y[r][c];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    double s = y[c];
#pragma unroll
    for (int q = 0; q < c; ++q) s -= Dg[c][q] * y[q];
    y[c] = s * rdiag[c];
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) Y[r][c] = y[c];
}

__global__ __launch_bounds__(256) void k_spd_inverse64(double* __restrict__ G,
                                                       double* __restrict__ Xb,
                                                       int32_t* __restrict__ fail) {
  constexpr int NB = 32;
  constexpr int64_t mp = 64;
  __shared__ double D0[NB][NB + 1], D1[NB][NB + 1], Y[NB][NB + 1];
  __shared__ double X0[NB][NB + 1], X1[NB][NB + 1], T0[NB][NB + 1];
  __shared__ double rd0[NB], rd1[NB];
  const int t = threadIdx.x;
  load_tile<NB>(D0, G, mp, 0, 0);
  load_tile<NB>(Y, G, mp, NB, 0);
  load_tile<NB>(D1, G, mp, NB, NB);
  __syncthreads();
  // step 0: L00, then X00 (wave 0) and L10 = G10 L00^{-T} (wave 1)
  chol_factor_block(D0, rd0, fail);
  if (t < NB) chol_inverse_block(D0, rd0, X0, t);
  if (t >= 64 && t < 64 + NB) chol_solve_row(D0, rd0, Y, t - 64);
  __syncthreads();
  // step 1: G11 - L10 L10^T, L11, X11
  {
    TileAcc<NB> td;
    td.mma_nt(Y, Y);
#pragma unroll
    for (int r = 0; r < 4; ++r) D1[td.row(r)][td.col()] -= td.acc[r];
  }
  __syncthreads();
  chol_factor_block(D1, rd1, fail);
  if (t < NB) chol_inverse_block(D1, rd1, X1, t);
  __syncthreads();
  // X10 = -X11 (L10 X00)
  {
    TileAcc<NB> tc;
    tc.mma_nn(Y, X0);
#pragma unroll
    for (int r = 0; r < 4; ++r) T0[tc.row(r)][tc.col()] = tc.acc[r];
  }
  __syncthreads();
  {
    TileAcc<NB> tx;
    tx.mma_nn(X1, T0);
    __syncthreads();  // every wave has read T0
#pragma unroll
    for (int r = 0; r < 4; ++r) T0[tx.row(r)][tx.col()] = -tx.acc[r];
  }
  __syncthreads();  // T0 = X10
  // L^{-1} out (the block above the diagonal is not written)
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    Xb[r + c * mp] = X0[r][c];
    Xb[(NB + r) + c * mp] = T0[r][c];
    Xb[(NB + r) + (NB + c) * mp] = X1[r][c];
  }
  // P = X^T X over G: P00 = X00^T X00 + X10^T X10, P10 = X11^T X10, P11 = X11^T X11
  {
    TileAcc<NB> p00, p10, p11;
    p00.mma_tn(X0, X0);
    p00.mma_tn(T0, T0);
    p10.mma_tn(X1, T0);
    p11.mma_tn(X1, X1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gi = p00.row(r), gj = p00.col();
      if (gi >= gj) {
        G[gi + gj * mp] = p00.acc[r];
        G[gj + gi * mp] = p00.acc[r];
      }
      const int64_t hi = NB + p10.row(r), hj = p10.col();
      G[hi + hj * mp] = p10.acc[r];
      G[hj + hi * mp] = p10.acc[r];
      const int64_t ki = NB + p11.row(r), kj = NB + p11.col();
      if (ki >= kj) {
        G[ki + kj * mp] = p11.acc[r];
        G[kj + ki * mp] = p11.acc[r];
      }
    }
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
  for (int j0 = ai; j0 < half; j0 += kTileAhead) {
    TileRegs<NB> ra[kTileAhead], rb[kTileAhead];
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (j0 + d < half) {
        const int64_t J0 = (int64_t)(a0 + j0 + d) * NB;
        ra[d].load(G, mp, R0, J0);   // L_(b0+bi),(a0+j)
        rb[d].load(Xb, mp, J0, C0);  // X_(a0+j),(a0+ai)
      }
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (j0 + d < half) {
        __syncthreads();
        ra[d].store(At);
        rb[d].store(Bt);
        __syncthreads();
        ta.mma_nn(At, Bt);
      }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Ct[(R0 + ta.row(r)) + (C0 + ta.col()) * mp] = ta.acc[r];
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
  for (int j0 = 0; j0 <= bi; j0 += kTileAhead) {
    TileRegs<NB> ra[kTileAhead], rb[kTileAhead];
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (j0 + d <= bi) {
        const int64_t J0 = (int64_t)(b0 + j0 + d) * NB;
        ra[d].load(Xb, mp, R0, J0);  // X_(b0+bi),(b0+j)
        rb[d].load(Ct, mp, J0, C0);  // C_(b0+j),(a0+ai)
      }
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (j0 + d <= bi) {
        __syncthreads();
        ra[d].store(At);
        rb[d].store(Bt);
        __syncthreads();
        ta.mma_nn(At, Bt);
      }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Xb[(R0 + ta.row(r)) + (C0 + ta.col()) * mp] = -ta.acc[r];
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
  for (int l0 = bi; l0 < T; l0 += kTileAhead) {
    TileRegs<NB> ra[kTileAhead], rb[kTileAhead];
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (l0 + d < T) {
        const int64_t L0 = (int64_t)(l0 + d) * NB;
        ra[d].load(Xb, mp, L0, I0);  // X_li
        rb[d].load(Xb, mp, L0, J0);  // X_lj
      }
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (l0 + d < T) {
        __syncthreads();
        ra[d].store(At);
        rb[d].store(Bt);
        __syncthreads();
        ta.mma_tn(At, Bt);
      }
  }
  // on a diagonal tile only i >= j is written (with its mirror): one writer
  // per entry
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t gi = I0 + ta.row(r), gj = J0 + ta.col();
    if (bi != bj || gi >= gj) {
      G[gi + gj * mp] = ta.acc[r];
      G[gj + gi * mp] = ta.acc[r];
    }
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
  for (int k0 = 0; k0 <= bi; k0 += kTileAhead) {
    TileRegs<NB> ra[kTileAhead], rb[kTileAhead];
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (k0 + d <= bi) {
        const int64_t K0 = (int64_t)(k0 + d) * NB;
        ra[d].load(X, mp, I0, K0);
        rb[d].load_masked(In, ldin, K0, J0, nrows, ncols);
      }
#pragma unroll
    for (int d = 0; d < kTileAhead; ++d)
      if (k0 + d <= bi) {
        __syncthreads();
        ra[d].store(At);
        rb[d].store(Bt);
        __syncthreads();
        ta.mma_nn(At, Bt);
      }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t gi = I0 + ta.row(r), gj = J0 + ta.col();
    if (gi < nrows_out && gj < ncols) Out[gi + gj * ldout] = ta.acc[r];
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
  int64_t cps = (w + ksplit - 1) / ksplit;
  cps = (cps + 15) / 16 * 16;
  if (mp <= 256) {  // 64 x 64 tiles: less padding and more workgroups for small m
    const int T = (int)((mp + 63) / 64);
    hipLaunchKernelGGL(k_gram<64>, dim3(T * (T + 1) / 2, ksplit), dim3(256), 0, st, B, ldb, m, w,
                       Gpart, mp, cps);
    return;
  }
  const int T = (int)((mp + kRT - 1) / kRT);
  hipLaunchKernelGGL(k_gram<kRT>, dim3(T * (T + 1) / 2, ksplit), dim3(256), 0, st, B, ldb, m, w,
                     Gpart, mp, cps);
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
  if (mp == 2 * kNb) {
    hipLaunchKernelGGL(k_spd_inverse64, dim3(1), dim3(256), 0, st, G, Xb, fail);
    return;
  }
  const int T = (int)(mp / kNb);
  for (int k = 0; k < T; ++k) {
    const int rest = T - k - 1;
    const int tiles = k > 0 ? rest * (rest + 1) / 2 : 0;  // step k-1's update right of block k
    hipLaunchKernelGGL(k_chol_step<kNb>, dim3(rest + 1 + tiles), dim3(256), 0, st, G, Xb, mp, k,
                       T, fail);
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
