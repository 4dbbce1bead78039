// The normal-equation product out = A D^2 A^T u (the operator of eq. "normal")
// on the caller's own A and D^2, with no handle and no allocation, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops).  It runs the kernels of normal_matvec: the fused column pass
// (one read of A) and the fixed-order sum of its per-workgroup partials.  The
// partials and a zero-padded copy of u live in `scratch`, a static device
// array that each device holds until the process ends.
#include <stdint.h>

#include <mutex>
#include <string>

#include "common.h"

using namespace skipm;

namespace {

// Largest partial-sum block of a COL_NORMAL pass: at most 512 workgroups (the
// 256-thread shapes) of one partial each, of at most kMaxM rows; then the
// padded u (kMaxM entries).
constexpr int64_t kMaxParts = 512;
constexpr int64_t kScratchDoubles = kMaxParts * kMaxM + kMaxM;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// This device's address of `scratch`, looked up once per device with that
// device current.  Host code uses only this address, never the array's name.
int scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the scratch table");
    return SKIPM_EDEVICE;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return SKIPM_EDEVICE;
    }
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return SKIPM_OK;
}

int64_t round_up64(int64_t a) { return (a + 63) / 64 * 64; }

}  // namespace

extern "C" int normal_matvec_noalloc(const void* A, int32_t a_dtype, int64_t m, int64_t n,
                                     int64_t lda, const double* d2, const double* u, double* out,
                                     hipStream_t st) {
  if (!A || !u || !out) return set_error("null argument"), SKIPM_EINVAL;
  if (a_dtype != SKIPM_F64 && a_dtype != SKIPM_F32)
    return set_error("a_dtype must be SKIPM_F64 or SKIPM_F32"), SKIPM_EINVAL;
  if (m < 1 || m > kMaxM || n < 1) return set_error("need 1 <= m <= 2048 and n >= 1"), SKIPM_EINVAL;
  if (lda < m || lda > kMaxM || lda % 4 != 0)
    return set_error("need m <= lda <= 2048 with lda a multiple of 4"), SKIPM_EINVAL;
  if (((uintptr_t)A & 15) != 0) return set_error("A must be 16-byte aligned"), SKIPM_EINVAL;
  const int nblk = colpass_nblk(lda, n, a_dtype, SKIPM_F64, COL_NORMAL);
  const int64_t lu = round_up64(lda), ldp = round_up64(m);
  if ((int64_t)nblk > kMaxParts || (int64_t)nblk * ldp + lu > kScratchDoubles)
    return set_error("shape needs more than the static scratch buffer"), SKIPM_EINVAL;
  int dev = 0;
  SK_CHECK_HIP(hipGetDevice(&dev));
  double* base = nullptr;
  SK_TRY(scratch_address(dev, &base));
  double* part = base;
  double* su = base + kMaxParts * kMaxM;
  // u, zero-padded to every row the pass reads (rows past m multiply A's
  // padding rows, which must be finite)
  launch_pad_copy_f64(su, lu, u, m, m, 1, st);
  ColPass cp{};
  cp.mode = COL_NORMAL;
  cp.A = A;
  cp.ta = a_dtype;
  cp.tc = SKIPM_F64;
  cp.lda = lda;
  cp.m = m;
  cp.n = n;
  cp.u = su;
  cp.d2 = d2;
  cp.part = part;
  cp.ldp = ldp;
  cp.nblk = nblk;
  cp.nt = lda * n * (a_dtype == SKIPM_F64 ? 8 : 4) > kStreamBytes ? 1 : 0;
  if (launch_colpass(cp, st) != 0) return set_error("no column-pass kernel for this shape"), SKIPM_EINVAL;
  launch_finish(part, ldp, 0, nblk, m, 1.0, nullptr, 0.0, out, nullptr, st);
  SK_CHECK_HIP(hipGetLastError());
  return SKIPM_OK;
}
