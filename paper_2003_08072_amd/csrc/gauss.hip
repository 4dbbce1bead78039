// Gaussian sketching matrix W_G (Sec. 5; the paper's experiments use it) for
// dense A.  W_G (n x w, N(0, 1) entries from a counter-based generator) is
// written already scaled by D, Wd = D W_G, so that the sketch is one GEMM,
// B = A Wd (k_gauss_gemm, FP64 on the matrix cores, split along n), and the
// correction vector's W t is one GEMV, (W_G t)_j = (Wd t)_j / d_j
// (k_gauss_gemv).
//
// Entries (j, c), (j, c + 1), c even, with salt k (one Box-Muller pair; the
// same definition as the reference generator):
//   base = mix(seed + G (1 + k)), q = jw + c, h1 = mix(base ^ 2q), h2 = mix(base ^ (2q + 1))
//   u1 = ((h1 >> 11) + 1) 2^-53, u2 = (h2 >> 11) 2^-53, r = sqrt(-2 ln u1), t = 2 pi u2
//   W_jc = r cos t, W_j,c+1 = r sin t, each rounded to an 8-bit significand (ties to even)
#include "common.h"

namespace skipm {

namespace {

__device__ __forceinline__ uint64_t gmix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ double round8(double z) {
  int e = 0;
  const double m = frexp(z, &e);
  return ldexp(rint(ldexp(m, 8)), e - 8);
}

// Wd[j + c ldw] = d_j W_G[j, c].  Thread j of the x grid owns row j (coalesced
// stores down each column) and kFillPairs column pairs per y block, so no
// index division; sin(2 pi u2), cos(2 pi u2) come from one sincospi of 2 u2
// (2 u2 is exact), which needs no range reduction of a rounded 2 pi u2.
constexpr int kFillPairs = 8;

__global__ __launch_bounds__(256) void k_gauss_fill(uint64_t base, int64_t n, int64_t w,
                                                    const double* __restrict__ dscale, int is_d2,
                                                    double* __restrict__ Wd, int64_t ldw) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double dj = is_d2 ? sqrt(dscale[j]) : dscale[j];
  const int64_t npair = (w + 1) / 2;
  const uint64_t row = (uint64_t)j * (uint64_t)w;
  for (int64_t p0 = (int64_t)blockIdx.y * kFillPairs; p0 < npair;
       p0 += (int64_t)gridDim.y * kFillPairs) {
    const int64_t p1 = p0 + kFillPairs < npair ? p0 + kFillPairs : npair;
    for (int64_t cp = p0; cp < p1; ++cp) {
      const int64_t c = 2 * cp;
      const uint64_t q = row + (uint64_t)c;
      const uint64_t h1 = gmix(base ^ (2 * q));
      const uint64_t h2 = gmix(base ^ (2 * q + 1));
      const double u1 = ((double)(h1 >> 11) + 1.0) * 0x1.0p-53;
      const double u2 = (double)(h2 >> 11) * 0x1.0p-53;
      const double r = sqrt(-2.0 * log(u1));
      double sn, cs;
      sincospi(2.0 * u2, &sn, &cs);
      Wd[j + c * ldw] = dj * round8(r * cs);
      if (c + 1 < w) Wd[j + (c + 1) * ldw] = dj * round8(r * sn);
    }
  }
}

// ---------------------------------------------------------------------------
// B_s = A[:, K_s] Wd[K_s, :] for the K slices K_s of [0, n) (slice s covers
// [s kc, (s + 1) kc), the last one up to n), FP64 on the matrix cores.
//
// One workgroup of four waves per 128 x 128 output tile and slice; each wave
// owns a 64 x 64 quarter as 4 x 4 blocks of 16 x 16.  Per stage of 16 values
// of k, the 128 x 16 panel of A and the 16 x 128 panel of Wd go through LDS
// (two buffers: the next stage's loads are in flight in registers while this
// stage's 64 MFMAs run, one barrier per stage).  v_mfma_f64_16x16x4 takes, in
// lane l, A[l%16][l/16] of a 16 x 4 block and B[l/16][l%16] of a 4 x 16 block
// and accumulates D[l/16 + 4r][l%16] in element r of a four-double register.
// Every output element is a sum over k in increasing order within its slice.
// In LDS the Wd panel keeps its columns (k contiguous, odd pitch): its stores
// and the MFMA operand reads both stay free of bank conflicts.
// ---------------------------------------------------------------------------
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef double dacc4 __attribute__((ext_vector_type(4)));
constexpr int kGT = 128;  // output tile
constexpr int kGK = 16;   // k per stage
constexpr int kGP = kGT + 2;  // LDS row pitch of the A panel (16-byte aligned rows)
constexpr int kWP = kGK + 1;  // LDS pitch of a Wd panel column (k contiguous)

__global__ __launch_bounds__(256) void k_gauss_gemm(const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ W, int64_t ldw,
                                                    int64_t w, int64_t n, int64_t kc,
                                                    double* __restrict__ out, int64_t lw) {
  __shared__ double As[2][kGK][kGP];
  __shared__ double Bs[2][kGT][kWP];
  const int tiles_r = (int)((lda + kGT - 1) / kGT);
  const int tr = blockIdx.x % tiles_r, tc = blockIdx.x / tiles_r;
  const int slice = blockIdx.y;
  const int64_t i0 = (int64_t)tr * kGT, c0 = (int64_t)tc * kGT;
  const int64_t kb = (int64_t)slice * kc;
  const int64_t ke = slice + 1 == (int)gridDim.y ? n : kb + kc;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  // load mapping: A panel, 4 x (one column kk, rows 2 rp, 2 rp + 1);
  // Wd panel, 4 x (one column cc, k = 2 kp, 2 kp + 1)
  const int a_kk = t >> 6, a_rp = t & 63;
  const int w_cc = t >> 3, w_kp = t & 7;
  const bool a_row_ok = i0 + 2 * a_rp < lda;  // lda is even, so the pair is in or out
  dvec2 ra[4], rw[4];
  auto fetch = [&](const int64_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t k = k0 + a_kk + 4 * q;
      ra[q] = (dvec2)0.0;
      if (a_row_ok && k < ke) ra[q] = *(const dvec2*)(A + k * lda + i0 + 2 * a_rp);
      const int64_t c = c0 + w_cc + 32 * q;
      const int64_t kw = k0 + 2 * w_kp;
      rw[q] = (dvec2)0.0;
      if (c < w) {
        const double* pw = W + c * ldw + kw;
        if (kw + 1 < ke) {
          rw[q] = *(const dvec2*)pw;
        } else if (kw < ke) {
          rw[q].x = pw[0];
        }
      }
    }
  };
  auto stash = [&](const int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *(dvec2*)&As[b][a_kk + 4 * q][2 * a_rp] = ra[q];
      Bs[b][w_cc + 32 * q][2 * w_kp] = rw[q].x;
      Bs[b][w_cc + 32 * q][2 * w_kp + 1] = rw[q].y;
    }
  };
  dacc4 acc[4][4];
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = (dacc4)0.0;
  const int64_t nst = (ke - kb + kGK - 1) / kGK;
  fetch(kb);
  stash(0);
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int b = (int)(st & 1);
    if (st + 1 < nst) fetch(kb + (st + 1) * kGK);
#pragma unroll
    for (int s4 = 0; s4 < kGK / 4; ++s4) {
      double fa[4], fb[4];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) fa[ib] = As[b][4 * s4 + lk][64 * wr + 16 * ib + li];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) fb[jb] = Bs[b][64 * wc + 16 * jb + li][4 * s4 + lk];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[ib], fb[jb], acc[ib][jb], 0, 0, 0);
    }
    if (st + 1 < nst) stash(b ^ 1);
    __syncthreads();
  }
  double* o = out + (int64_t)slice * lw;
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const int64_t c = c0 + 64 * wc + 16 * jb + li;
      if (c >= w) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 64 * wr + 16 * ib + lk + 4 * r;
        if (i < lda) o[c * lda + i] = acc[ib][jb][r];
      }
    }
}

// gy_j = sum over c of Wd[j, c] t_c (c in increasing order): one thread per
// row j, so every load of a column is one coalesced run across the wave.
__global__ __launch_bounds__(128) void k_gauss_gemv(const double* __restrict__ W, int64_t ldw,
                                                    int64_t n, int64_t w,
                                                    const double* __restrict__ t,
                                                    double* __restrict__ gy) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double* p = W + j;
  double acc = 0.0;
  int64_t c = 0;
  for (; c + 8 <= w; c += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = p[(c + q) * ldw];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += v[q] * t[c + q];
  }
  for (; c < w; ++c) acc += p[c * ldw] * t[c];
  gy[j] = acc;
}

// out[i] = sum over s of part[s lw + i], s in order
__global__ __launch_bounds__(256) void k_sum_slices(const double* __restrict__ part, int ns,
                                                    int64_t lw, double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lw; i += stride) {
    double s = 0;
    for (int q = 0; q < ns; ++q) s += part[(int64_t)q * lw + i];
    out[i] = s;
  }
}

}  // namespace

void launch_gauss_gemm(const double* A, int64_t lda, const double* Wd, int64_t ldw, int64_t w,
                       int64_t n, int ns, double* out, hipStream_t st) {
  const int64_t tiles = ((lda + kGT - 1) / kGT) * ((w + kGT - 1) / kGT);
  // slices of a multiple of 16 values of k (the last one takes the rest)
  int64_t kc = (n / ns) / kGK * kGK;
  if (kc < kGK) kc = kGK;
  int used = (int)((n + kc - 1) / kc);
  if (used > ns) used = ns;
  hipLaunchKernelGGL(k_gauss_gemm, dim3((unsigned)tiles, (unsigned)used), dim3(256), 0, st, A, lda,
                     Wd, ldw, w, n, kc, out, lda * w);
}

int gauss_gemm_slices(int64_t n, int ns) {
  int64_t kc = (n / ns) / kGK * kGK;
  if (kc < kGK) kc = kGK;
  const int64_t used = (n + kc - 1) / kc;
  return (int)(used < ns ? used : ns);
}

void launch_gauss_gemv(const double* Wd, int64_t ldw, int64_t n, int64_t w, const double* t,
                       double* gy, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gauss_gemv, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, Wd, ldw, n,
                     w, t, gy);
}

void launch_sum_slices(const double* part, int ns, int64_t lw, double* out, hipStream_t st) {
  int64_t blocks = (lw + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)blocks), dim3(256), 0, st, part, ns, lw, out);
}

void launch_gauss_fill(uint64_t seed, int64_t k, int64_t n, int64_t w, const double* dscale,
                       int is_d2, double* Wd, int64_t ldw, hipStream_t st) {
  // base = mix(seed + G (1 + k)), on the host (mod 2^64)
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(1 + k);
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  if (n <= 0 || w <= 0) return;
  const int64_t bx = (n + 255) / 256;
  int64_t by = ((w + 1) / 2 + kFillPairs - 1) / kFillPairs;
  if (by > 65535) by = 65535;  // the y loop covers the rest
  hipLaunchKernelGGL(k_gauss_fill, dim3((unsigned)bx, (unsigned)by), dim3(256), 0, st, z, n, w,
                     dscale, is_d2, Wd, ldw);
}

// Number of K slices for B = A Wd: the GEMM's 128 x 128 output tiles times the
// slices is the workgroup count, and with T tiles on 256 CUs the last round
// of workgroups runs on T s mod 256 CUs only.  Take the s (at most 32, slices
// of at least 1024 columns) whose workgroups fill the rounds best, T s / (256
// ceil(T s / 256)), among those with at least 512 workgroups (two per CU) when
// there are such; ties go to the fewer slices (less to sum afterwards).
int gauss_ksplit(int64_t lda, int64_t w, int64_t n) {
  const int64_t tiles = ((lda + 127) / 128) * ((w + 127) / 128);
  int64_t smax = n / 1024;
  if (smax > 32) smax = 32;
  if (smax <= 1 || tiles <= 0) return 1;
  const bool can_fill = tiles * smax >= 512;
  int best = 1;
  double best_eff = -1.0;
  for (int64_t s = 1; s <= smax; ++s) {
    const int64_t wg = tiles * s;
    if (can_fill && wg < 512) continue;
    const double eff = (double)wg / (256.0 * (double)((wg + 255) / 256));
    if (eff > best_eff + 1e-12) {
      best_eff = eff;
      best = (int)s;
    }
  }
  return best;
}

}  // namespace skipm
