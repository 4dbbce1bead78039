// Gaussian sketching matrix W_G (Sec. 5; the paper's experiments use it) for
// dense A.  W_G (n x w, N(0, 1) entries from a counter-based generator) is
// written already scaled by D, Wd = D W_G, so that the sketch is one plain
// GEMM, B = A Wd (rocBLAS, FP64 on the matrix cores), and the correction
// vector's W t is one GEMV, (W_G t)_j = (Wd t)_j / d_j.
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
