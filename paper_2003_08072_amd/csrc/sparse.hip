// Sparse (CSR) constraint matrices.  The library keeps A twice:
//   CSR (row pointers, column indices, values) for products A v, and
//   CSC (column pointers, row indices, values), built once on the device, for
//   the column dots a_j^T u of A^T u and for the bucket-gathered sketch.
// A fused pass of the dense path (one read of each column doing both the dot
// and the axpy) becomes two passes here:
//   k_csc_dot   per column j: t_j = a_j^T u, then the mode's per-column work
//               (r_d, d^2, the coefficients of A x and A(sigma mu/s + d^2 r_d);
//               or d^2 t for A D^2 A^T u; or ds for the epilogue)
//   k_csr_seg   y = A coef: rows are cut into segments of at most kSeg
//               non-zeros (the all-ones row of the workloads has n of them), one
//               wave sums one segment in a fixed order
//   k_csr_fold  one wave per row adds the row's segment sums in order
// No floating-point atomics anywhere, so every result is bitwise reproducible.
#include "common.h"

namespace skipm {

namespace {

constexpr int kMaxRowsLds = (int)kMaxM;

__device__ __forceinline__ double wsum(double v) { return lane_group_sum<64>(v); }

// rowptr monotone from 0 to nnz, column indices in range and strictly
// increasing inside each row.  One thread per row.
// One wave per row: row pointers in range and monotone, columns in range and
// strictly increasing along the row.
__global__ __launch_bounds__(256) void k_csr_check(const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colidx,
                                                   int64_t m, int64_t n, int64_t nnz,
                                                   int32_t* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < m; i += nwaves) {
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    if ((i == 0 && b != 0) || b < 0 || e < b || e > nnz || (i == m - 1 && e != nnz)) {
      if (lane == 0) atomicOr(bad, 1);
      continue;
    }
    int flag = 0;
    for (int64_t k = b + lane; k < e; k += 64) {
      const int64_t c = colidx[k];
      if (c < 0 || c >= n || (k > b && c <= (int64_t)colidx[k - 1])) flag = 1;
    }
    if (flag) atomicOr(bad, 2);
  }
}

__device__ __forceinline__ int64_t row_of(const int32_t* __restrict__ rowptr, int64_t m,
                                          int64_t k) {
  // largest i with rowptr[i] <= k (rows may be empty)
  int64_t lo = 0, hi = m;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (rowptr[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_col_count(const int32_t* __restrict__ colidx,
                                                   int64_t nnz, int32_t* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride)
    atomicAdd(&cnt[colidx[k]], 1);
}

template <typename TV>
__global__ __launch_bounds__(256) void k_csc_fill(const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colidx,
                                                  const TV* __restrict__ val, int64_t m,
                                                  int64_t nnz, const int32_t* __restrict__ colptr,
                                                  int32_t* __restrict__ cursor,
                                                  int32_t* __restrict__ rowidx,
                                                  TV* __restrict__ cval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
    const int32_t c = colidx[k];
    const int64_t pos = colptr[c] + atomicAdd(&cursor[c], 1);
    rowidx[pos] = (int32_t)row_of(rowptr, m, k);
    cval[pos] = val[k];
  }
}

// insertion sort of each column's (row, value) pairs by row (one thread per column)
template <typename TV>
__global__ __launch_bounds__(256) void k_csc_sort(const int32_t* __restrict__ colptr, int64_t n,
                                                  int32_t* __restrict__ rowidx,
                                                  TV* __restrict__ cval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    const int64_t b = colptr[j], e = colptr[j + 1];
    for (int64_t k = b + 1; k < e; ++k) {
      const int32_t r = rowidx[k];
      const TV v = cval[k];
      int64_t q = k - 1;
      while (q >= b && rowidx[q] > r) {
        rowidx[q + 1] = rowidx[q];
        cval[q + 1] = cval[q];
        --q;
      }
      rowidx[q + 1] = r;
      cval[q + 1] = v;
    }
  }
}

// Segments: row i covers ceil(len_i / kSeg) consecutive segments (at least one).
__global__ __launch_bounds__(256) void k_seg_count(const int32_t* __restrict__ rowptr, int64_t m,
                                                  int seg, int32_t* __restrict__ nseg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const int64_t len = rowptr[i + 1] - rowptr[i];
    nseg[i] = (int32_t)(len > 0 ? (len + seg - 1) / seg : 1);
  }
}

__global__ __launch_bounds__(256) void k_seg_fill(const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ segptr, int64_t m,
                                                  int seg, int32_t* __restrict__ seg_start,
                                                  int32_t* __restrict__ seg_end) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int64_t b = rowptr[i], e = rowptr[i + 1];
  int64_t s = segptr[i];
  for (int64_t k = b; k < e || k == b; k += seg, ++s) {
    seg_start[s] = (int32_t)k;
    seg_end[s] = (int32_t)(k + seg < e ? k + seg : e);
    if (e == b) break;
  }
}

struct CscArgs {
  const int32_t* colptr;
  const int32_t* rowidx;
  const void* cval;
  int64_t m, n;
  const double* u;
  const double* x;
  const double* s;
  const double* c;
  const double* rd;
  const double* d2;
  double* coef1;   // NORMAL / EPILOGUE: d2 t ; PROLOGUE: x (not written, read from x) ; DOT: t
  double* coef2;   // PROLOGUE: sigma mu / s + d2 r_d
  double* rd_out;
  double* d2_out;
  double* ds_out;
  double* red;
  const double* sc;
  const int32_t* done;
  CgFuse cg;  // COL_NORMAL inside CG: open the iteration (stop test, beta, d_k)
};

template <typename TV, int MODE>
__global__ __launch_bounds__(256) void k_csc_dot(CscArgs a) {
  __shared__ double us[kMaxRowsLds];
  __shared__ double sred[4][2];
  const int lane = threadIdx.x & 63;
  const bool cg_open = MODE == COL_NORMAL && a.cg.on && a.cg.k > 0;
  // Everything the pass starts from is requested before the done flag is
  // read, so that the start waits one memory latency: the range of the
  // thread's first column, the m-vector entries it stages into LDS (u, or z_k
  // and d_{k-1} when a CG iteration opens), and the partial sums r^T z, r^T r
  // (wave 0; up to kPre per lane, any further ones in a loop below).  Every
  // index is clamped in bounds; clamped values are never used.
  const int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j0c = j0 < a.n ? j0 : a.n - 1;
  const int64_t cb0 = a.colptr[j0c], ce0 = a.colptr[j0c + 1];
  // (the first kSt * 256 rows; rows beyond are staged in a loop below)
  constexpr int kSt = 4;
  double st0[kSt], st1[kSt];
#pragma unroll
  for (int q = 0; q < kSt; ++q) {
    const int64_t i = threadIdx.x + 256 * q;
    const int64_t ic = i < a.m ? i : 0;
    if (cg_open) {
      st0[q] = a.cg.z[ic];
      st1[q] = a.cg.d_old[ic];
    } else {
      st0[q] = a.u[ic];
    }
  }
  // wave 0 of a pass that opens a CG iteration requests the partial sums
  // (up to kPre per lane; any further ones in a loop) before it reads the
  // done flag, and sums them in the order p = lane, lane + 64, ..., then over
  // the wave: the same sums in the same order in every workgroup, hence the
  // same decision
  if (cg_open && threadIdx.x < 64) {
    constexpr int kPre = 4;
    const int pn = a.cg.np;
    double pre0[kPre], pre1[kPre];
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int p = lane + 64 * q;
      const int pc = p < pn ? p : pn - 1;
      pre0[q] = a.cg.prz[2 * (int64_t)pc];
      pre1[q] = a.cg.prz[2 * (int64_t)pc + 1];
    }
    if (a.done && *a.done) return;
    double s0 = 0, s1 = 0;
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const bool in = lane + 64 * q < pn;
      s0 += in ? pre0[q] : 0.0;
      s1 += in ? pre1[q] : 0.0;
    }
    for (int p = lane + 64 * kPre; p < pn; p += 64) {
      s0 += a.cg.prz[2 * p];
      s1 += a.cg.prz[2 * p + 1];
    }
    s0 = lane_group_sum<64>(s0);
    s1 = lane_group_sum<64>(s1);
    if (lane == 0) {
      sred[0][0] = s0;
      sred[0][1] = s1;
    }
  }
  if (a.done && *a.done) return;
  if (cg_open) {
    __syncthreads();
    const int64_t k = a.cg.k;
    double* sc = a.cg.sc;
    int32_t* is = a.cg.is;
    const double rz = sred[0][0], rr = sred[0][1];
    const double crit = is[I_CG_RESID] ? rr : rz;
    const bool stop = k >= is[I_CG_MAX] || crit <= sc[S_CG_TOL2] || !(rz > 0);
    const double beta =
        a.cg.inner == SKIPM_INNER_CG ? rz / sc[S_CG_RZH0 + (int)((k - 1) & 1)] : 0.0;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[S_CG_RZ] = rz;
      sc[S_V_RR] = rr;
      sc[S_CG_RZH0 + (int)(k & 1)] = rz;
      is[I_CG_ITERS] = (int32_t)k;
      if (stop) is[I_CG_DONE] = 1;
    }
    if (stop) return;
#pragma unroll
    for (int q = 0; q < kSt; ++q) {
      const int64_t i = threadIdx.x + 256 * q;
      if (i < a.m) {
        const double di = st0[q] + beta * st1[q];
        us[i] = di;
        if (blockIdx.x == 0) a.cg.d_new[i] = di;
      }
    }
    for (int64_t i = threadIdx.x + 256 * kSt; i < a.m; i += 256) {
      const double di = a.cg.z[i] + beta * a.cg.d_old[i];
      us[i] = di;
      if (blockIdx.x == 0) a.cg.d_new[i] = di;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kSt; ++q) {
      const int64_t i = threadIdx.x + 256 * q;
      if (i < a.m) us[i] = st0[q];
    }
    for (int64_t i = threadIdx.x + 256 * kSt; i < a.m; i += 256) us[i] = a.u[i];
  }
  __syncthreads();
  const TV* __restrict__ cv = (const TV*)a.cval;
  double mu = 0, sigma = 0;
  if (MODE == COL_PROLOGUE) {
    mu = a.sc[S_MU];
    sigma = a.sc[S_SIGMA];
  }
  double r0 = 0, r1 = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t cb = cb0, ce = ce0;
  for (int64_t j = j0; j < a.n; j += stride) {
    // the next column's range is requested before this column is summed
    const int64_t jn = j + stride < a.n ? j + stride : a.n - 1;
    const int64_t nb = a.colptr[jn], ne = a.colptr[jn + 1];
    const int64_t b = cb, e = ce;
    cb = nb;
    ce = ne;
    double t = 0;
    for (int64_t k = b; k < e; ++k) t += (double)cv[k] * us[a.rowidx[k]];
    if (MODE == COL_NORMAL) {
      a.coef1[j] = a.d2 ? a.d2[j] * t : t;
    } else if (MODE == COL_DOT) {
      a.coef1[j] = t;
    } else if (MODE == COL_EPILOGUE) {
      a.ds_out[j] = -a.rd[j] - t;
      a.coef1[j] = a.d2[j] * t;
    } else {  // COL_PROLOGUE
      const double xj = a.x[j], sj = a.s[j], cj = a.c[j];
      const double rdj = t + sj - cj;
      const double d2j = xj / sj;
      a.rd_out[j] = rdj;
      a.d2_out[j] = d2j;
      a.coef2[j] = sigma * mu / sj + d2j * rdj;
      r0 += rdj * rdj;
      r1 += cj * xj;
    }
  }
  if (MODE == COL_PROLOGUE) {
    r0 = wsum(r0);
    r1 = wsum(r1);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      sred[wid][0] = r0;
      sred[wid][1] = r1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t0 = 0, t1 = 0;
      for (int w = 0; w < 4; ++w) {
        t0 += sred[w][0];
        t1 += sred[w][1];
      }
      a.red[blockIdx.x * 8 + 0] = t0;
      a.red[blockIdx.x * 8 + 1] = t1;
      a.red[blockIdx.x * 8 + 2] = 0.0;
    }
  }
}

// One wave per segment: segsum[v][s] = sum over the segment of a_ik coef_v[k].
template <typename TV, int NV>
__global__ __launch_bounds__(256) void k_csr_seg(const int32_t* __restrict__ colidx,
                                                 const TV* __restrict__ val,
                                                 const int32_t* __restrict__ seg_start,
                                                 const int32_t* __restrict__ seg_end,
                                                 int64_t nseg, const double* __restrict__ coef1,
                                                 const double* __restrict__ coef2,
                                                 double* __restrict__ segsum,
                                                 const int32_t* __restrict__ done) {
  const int lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (s >= nseg) return;
  const int64_t b = seg_start[s], e = seg_end[s];  // requested before the done flag is read
  if (done && *done) return;
  double acc1 = 0, acc2 = 0;
  // four non-zeros per lane per trip: their indices and values are loaded
  // first, then the four gathers are in flight together; the products are
  // added in non-zero order
  constexpr int U = 4;
  for (int64_t k = b + lane; k < e; k += 64 * U) {
    int32_t c[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kk = k + 64 * u;
      c[u] = kk < e ? colidx[kk] : -1;
      v[u] = kk < e ? (double)val[kk] : 0.0;
    }
    double g1[U], g2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      g1[u] = c[u] >= 0 ? coef1[c[u]] : 0.0;
      if (NV > 1) g2[u] = c[u] >= 0 ? coef2[c[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (c[u] < 0) break;
      acc1 += v[u] * g1[u];
      if (NV > 1) acc2 += v[u] * g2[u];
    }
  }
  acc1 = wsum(acc1);
  if (NV > 1) acc2 = wsum(acc2);
  if (lane == 0) {
    segsum[s] = acc1;
    if (NV > 1) segsum[nseg + s] = acc2;
  }
}

// One wave per row: out[i] = scale * sum of the row's segment sums (in order) + beta * add[i];
// with dvec, also the workgroup's partial sum of dvec_i out_i (its four rows in order).
__global__ __launch_bounds__(256) void k_csr_fold(const double* __restrict__ segsum,
                                                  const int32_t* __restrict__ segptr, int64_t m,
                                                  double scale, const double* __restrict__ add,
                                                  double beta, double* __restrict__ out,
                                                  const double* __restrict__ dvec,
                                                  double* __restrict__ dq_out,
                                                  const int32_t* __restrict__ done) {
  __shared__ double dq[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + wid;
  const int64_t ic = i < m ? i : m - 1;
  const int64_t sb = segptr[ic], se = segptr[ic + 1];  // requested before the done flag is read
  if (done && *done) return;
  double v = 0;
  if (i < m) {
    const int64_t b = sb, e = se;
    double acc = 0;
    // eight loads in flight per lane (rows with many segments, such as a
    // dense row, would otherwise wait out one load latency per term); each
    // lane still adds its terms in segment order
    int64_t s = b + lane;
    for (; s + 7 * 64 < e; s += 8 * 64) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = segsum[s + 64 * q];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += t[q];
    }
    for (; s < e; s += 64) acc += segsum[s];
    acc = wsum(acc);
    v = scale * acc;
    if (add) v += beta * add[i];
    if (lane == 0) out[i] = v;
  }
  if (dvec) {  // uniform: every wave of the workgroup reaches the barrier
    if (lane == 0) dq[wid] = i < m ? dvec[i] * v : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) dq_out[blockIdx.x] = ((dq[0] + dq[1]) + dq[2]) + dq[3];
  }
}

// Sketch from CSC: one wave per bucket accumulates B[:, b] in LDS, column by
// column in item order (the lanes of one step touch distinct rows).  The
// items' metadata (column, coefficient, column range) and the first kHead
// entries of each item's column are fetched 64 items at a time, one item per
// lane, so a block of 64 columns waits out one load latency; the columns are
// then added one after another from registers (read across lanes), the
// entries past the first kHead of a longer column by strided loads.  The
// order of the additions is the plain item-by-item order.
constexpr int kHead = 4;
__device__ __forceinline__ float readlane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_val(double v, int l) { return readlane_f64(v, l); }

template <typename TV>
__global__ __launch_bounds__(256) void k_csc_sketch(const int32_t* __restrict__ colptr,
                                                    const int32_t* __restrict__ rowidx,
                                                    const TV* __restrict__ cval, int64_t m,
                                                    int64_t nnz,
                                                    int s, const double* __restrict__ dsc,
                                                    int is_d2, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ perm,
                                                    const int8_t* __restrict__ sign, int w,
                                                    double* __restrict__ B, int64_t ldb) {
  extern __shared__ double accs[];  // [4][ldb]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double* acc = accs + (int64_t)wid * ldb;
  const int bkt = blockIdx.x * 4 + wid;
  if (bkt >= w) return;
  for (int64_t i = lane; i < ldb; i += 64) acc[i] = 0.0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  const int beg = ptr[bkt], end = ptr[bkt + 1];
  const int64_t last = nnz > 0 ? nnz - 1 : 0;
  for (int it0 = beg; it0 < end; it0 += 64) {
    const int itl = it0 + lane;
    int32_t cb_l = 0, ce_l = 0;
    double coef_l = 0.0;
    if (itl < end) {
      const int item = perm[itl];
      const int64_t j = item / s;
      const double dj = dsc[j];
      coef_l = (double)sign[item] * (is_d2 ? sqrt(dj) : dj);
      cb_l = colptr[j];
      ce_l = colptr[j + 1];
    }
    // the first kHead entries of this lane's column (in-bounds indices past its end)
    int32_t hr[kHead];
    TV hv[kHead];
#pragma unroll
    for (int e = 0; e < kHead; ++e) {
      const int64_t k = (int64_t)cb_l + e;
      const int64_t kc = k < ce_l ? k : last;
      hr[e] = rowidx[kc];
      hv[e] = cval[kc];
    }
    const int cnt = end - it0 < 64 ? end - it0 : 64;
    for (int q = 0; q < cnt; ++q) {
      const int32_t cb = __builtin_amdgcn_readlane(cb_l, q);
      const int32_t ce = __builtin_amdgcn_readlane(ce_l, q);
      const double coef = readlane_f64(coef_l, q);
      // lane e < kHead adds entry cb + e of column q
      int32_t r0 = 0;
      TV v0 = 0;
#pragma unroll
      for (int e = 0; e < kHead; ++e) {
        const int32_t re = __builtin_amdgcn_readlane(hr[e], q);
        const TV ve = readlane_val(hv[e], q);
        if (lane == e) {
          r0 = re;
          v0 = ve;
        }
      }
      if (lane < kHead && cb + lane < ce) acc[r0] += coef * (double)v0;
      for (int64_t k = (int64_t)cb + kHead + lane; k < ce; k += 64)
        acc[rowidx[k]] += coef * (double)cval[k];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
  double* out = B + (int64_t)bkt * ldb;
  for (int64_t i = lane; i < ldb; i += 64) out[i] = acc[i];
}

unsigned grid_n(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void launch_csr_check(const int32_t* rowptr, const int32_t* colidx, int64_t m, int64_t n,
                      int64_t nnz, int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_csr_check, dim3(grid_n(m * 64)), dim3(256), 0, st, rowptr, colidx, m, n,
                     nnz, bad);
}

void launch_build_csc(const int32_t* rowptr, const int32_t* colidx, const void* val, int vdt,
                      int64_t m, int64_t n, int64_t nnz, int32_t* cnt, int32_t* colptr,
                      int32_t* cursor, int32_t* rowidx, void* cval, hipStream_t st) {
  launch_fill_i32(cnt, 0, n, st);
  hipLaunchKernelGGL(k_col_count, dim3(grid_n(nnz)), dim3(256), 0, st, colidx, nnz, cnt);
  launch_bucket_scan(cnt, colptr, cursor, (int)n, st);
  if (vdt == SKIPM_F64) {
    hipLaunchKernelGGL(k_csc_fill<double>, dim3(grid_n(nnz)), dim3(256), 0, st, rowptr, colidx,
                       (const double*)val, m, nnz, colptr, cursor, rowidx, (double*)cval);
    hipLaunchKernelGGL(k_csc_sort<double>, dim3(grid_n(n)), dim3(256), 0, st, colptr, n, rowidx,
                       (double*)cval);
  } else {
    hipLaunchKernelGGL(k_csc_fill<float>, dim3(grid_n(nnz)), dim3(256), 0, st, rowptr, colidx,
                       (const float*)val, m, nnz, colptr, cursor, rowidx, (float*)cval);
    hipLaunchKernelGGL(k_csc_sort<float>, dim3(grid_n(n)), dim3(256), 0, st, colptr, n, rowidx,
                       (float*)cval);
  }
}

void launch_build_segments(const int32_t* rowptr, int64_t m, int seg, int32_t* nseg,
                           int32_t* segptr, int32_t* cursor, int32_t* seg_start, int32_t* seg_end,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_seg_count, dim3(grid_n(m)), dim3(256), 0, st, rowptr, m, seg, nseg);
  launch_bucket_scan(nseg, segptr, cursor, (int)m, st);
  if (seg_start && seg_end)  // first call: counts and offsets only
    hipLaunchKernelGGL(k_seg_fill, dim3(grid_n(m)), dim3(256), 0, st, rowptr, segptr, m, seg,
                       seg_start, seg_end);
}

int launch_csc_dot(const SparseA& A, int mode, const double* u, const double* x, const double* s,
                   const double* c, const double* rd, const double* d2, double* coef1,
                   double* coef2, double* rd_out, double* d2_out, double* ds_out, double* red,
                   const double* sc, const int32_t* done, int nblk, hipStream_t st,
                   const CgFuse* cg) {
  CscArgs a{};
  if (cg) a.cg = *cg;
  a.colptr = A.colptr;
  a.rowidx = A.rowidx;
  a.cval = A.cval;
  a.m = A.m;
  a.n = A.n;
  a.u = u;
  a.x = x;
  a.s = s;
  a.c = c;
  a.rd = rd;
  a.d2 = d2;
  a.coef1 = coef1;
  a.coef2 = coef2;
  a.rd_out = rd_out;
  a.d2_out = d2_out;
  a.ds_out = ds_out;
  a.red = red;
  a.sc = sc;
  a.done = done;
  if (A.m > kMaxRowsLds) return -1;
#define SK_CSC(TV)                                                                          \
  switch (mode) {                                                                           \
    case COL_NORMAL:                                                                        \
      hipLaunchKernelGGL((k_csc_dot<TV, COL_NORMAL>), dim3(nblk), dim3(256), 0, st, a);     \
      break;                                                                                \
    case COL_PROLOGUE:                                                                      \
      hipLaunchKernelGGL((k_csc_dot<TV, COL_PROLOGUE>), dim3(nblk), dim3(256), 0, st, a);   \
      break;                                                                                \
    case COL_EPILOGUE:                                                                      \
      hipLaunchKernelGGL((k_csc_dot<TV, COL_EPILOGUE>), dim3(nblk), dim3(256), 0, st, a);   \
      break;                                                                                \
    case COL_DOT:                                                                           \
      hipLaunchKernelGGL((k_csc_dot<TV, COL_DOT>), dim3(nblk), dim3(256), 0, st, a);        \
      break;                                                                                \
    default:                                                                                \
      return -1;                                                                            \
  }
  if (A.vdt == SKIPM_F64) {
    SK_CSC(double)
  } else {
    SK_CSC(float)
  }
#undef SK_CSC
  return 0;
}

void launch_csr_segsum(const SparseA& A, const double* coef1, const double* coef2,
                       double* segsum, const int32_t* done, hipStream_t st) {
  const unsigned gs = (unsigned)((A.nseg + 3) / 4);
  const bool two = coef2 != nullptr;
  if (A.vdt == SKIPM_F64) {
    if (!two)
      hipLaunchKernelGGL((k_csr_seg<double, 1>), dim3(gs), dim3(256), 0, st, A.colidx,
                         (const double*)A.val, A.seg_start, A.seg_end, A.nseg, coef1, coef2,
                         segsum, done);
    else
      hipLaunchKernelGGL((k_csr_seg<double, 2>), dim3(gs), dim3(256), 0, st, A.colidx,
                         (const double*)A.val, A.seg_start, A.seg_end, A.nseg, coef1, coef2,
                         segsum, done);
  } else {
    if (!two)
      hipLaunchKernelGGL((k_csr_seg<float, 1>), dim3(gs), dim3(256), 0, st, A.colidx,
                         (const float*)A.val, A.seg_start, A.seg_end, A.nseg, coef1, coef2,
                         segsum, done);
    else
      hipLaunchKernelGGL((k_csr_seg<float, 2>), dim3(gs), dim3(256), 0, st, A.colidx,
                         (const float*)A.val, A.seg_start, A.seg_end, A.nseg, coef1, coef2,
                         segsum, done);
  }
}

void launch_csr_fold(const SparseA& A, const double* segsum, int which, double scale,
                     const double* add, double beta, double* out, const int32_t* done,
                     hipStream_t st, const double* dvec, double* dq_out) {
  const unsigned gm = (unsigned)csr_fold_nblk(A.m);
  hipLaunchKernelGGL(k_csr_fold, dim3(gm), dim3(256), 0, st, segsum + (int64_t)which * A.nseg,
                     A.segptr, A.m, scale, add, beta, out, dvec, dq_out, done);
}

int csr_fold_nblk(int64_t m) { return (int)((m + 3) / 4); }

void launch_sketch_csc(const SparseA& A, int s, const double* dscale, int is_d2,
                       const int32_t* ptr, const int32_t* perm, const int8_t* sign, int w,
                       double* B, int64_t ldb, hipStream_t st) {
  const size_t lds = (size_t)4 * ldb * sizeof(double);
  const unsigned g = (unsigned)((w + 3) / 4);
  if (A.vdt == SKIPM_F64)
    hipLaunchKernelGGL(k_csc_sketch<double>, dim3(g), dim3(256), lds, st, A.colptr, A.rowidx,
                       (const double*)A.cval, A.m, A.nnz, s, dscale, is_d2, ptr, perm, sign, w,
                       B, ldb);
  else
    hipLaunchKernelGGL(k_csc_sketch<float>, dim3(g), dim3(256), lds, st, A.colptr, A.rowidx,
                       (const float*)A.cval, A.m, A.nnz, s, dscale, is_d2, ptr, perm, sign, w,
                       B, ldb);
}

int csc_dot_nblk(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace skipm
