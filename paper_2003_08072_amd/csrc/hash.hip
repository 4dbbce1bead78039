// Sparse embedding W: counter-based hash of (row j, block r) to a bucket and a
// sign, and a deterministic bucket-major ordering of the items so that the
// sketch B = A D W can be formed by gathering whole columns per bucket (no
// floating-point atomics; the summation order inside a bucket is by item index).
//
// Construction (block CountSketch, Sec. 2's sparse embedding made concrete):
//   base_r = mix(seed + G * (1 + k*s + r)),  h = mix(base_r ^ j),
//   bucket = r*(w/s) + (((h >> 32) * (w/s)) >> 32),  sign = (h & 1) ? -1 : +1,
// with mix the SplitMix64 output function (Steele, Lea, Flood 2014) and
// G = 0x9E3779B97F4A7C15.
#include "common.h"

namespace skipm {

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kMaxS = 16;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

struct HashBases {
  uint64_t base[kMaxS];
};

__global__ __launch_bounds__(256) void k_hash(HashBases hb, int s, int64_t n, int blk,
                                              int32_t* __restrict__ bucket,
                                              int8_t* __restrict__ sign,
                                              int32_t* __restrict__ count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    for (int r = 0; r < s; ++r) {
      const uint64_t h = mix64(hb.base[r] ^ (uint64_t)j);
      const int b = r * blk + (int)(((h >> 32) * (uint64_t)blk) >> 32);
      bucket[j * s + r] = b;
      sign[j * s + r] = (h & 1ull) ? (int8_t)-1 : (int8_t)1;
      if (count) atomicAdd(&count[b], 1);
    }
  }
}

// Bucket counts without per-item global atomics: workgroup g hashes the
// items of its own contiguous range, counts them per bucket in LDS, then adds
// each non-zero count to the global count once (a few workgroups per bucket
// instead of every item).
constexpr int kLdsBuckets = 8192;  // w up to this takes the LDS-aggregated kernels
constexpr int kAggBlocks = 64;     // workgroups of 1024 threads for them

__global__ __launch_bounds__(1024) void k_hash_agg(HashBases hb, int s, int64_t n, int blk,
                                                   int w, int32_t* __restrict__ bucket,
                                                   int8_t* __restrict__ sign,
                                                   int32_t* __restrict__ count) {
  __shared__ int32_t cnt[kLdsBuckets];
  for (int b = threadIdx.x; b < w; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int64_t nitems = n * s;
  const int64_t per = (nitems + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < nitems ? i0 + per : nitems;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int64_t j = i / s;
    const int r = (int)(i - j * s);
    const uint64_t h = mix64(hb.base[r] ^ (uint64_t)j);
    const int b = r * blk + (int)(((h >> 32) * (uint64_t)blk) >> 32);
    bucket[i] = b;
    sign[i] = (h & 1ull) ? (int8_t)-1 : (int8_t)1;
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < w; b += blockDim.x)
    if (cnt[b]) atomicAdd(&count[b], cnt[b]);
}

// Exclusive scan of the bucket counts (single workgroup), ptr has w+1 entries.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ count,
                                               int32_t* __restrict__ ptr,
                                               int32_t* __restrict__ cursor, int w) {
  __shared__ int32_t carry_s;
  __shared__ int32_t wsum[16];
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int base = 0; base < w; base += 1024) {
    const int i = base + threadIdx.x;
    const int32_t v = i < w ? count[i] : 0;
    // inclusive scan inside the wave
    int32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int32_t before = carry_s;
    for (int q = 0; q < wid; ++q) before += wsum[q];
    if (i < w) {
      ptr[i] = before + x - v;
      cursor[i] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t t = 0;
      for (int q = 0; q < 16; ++q) t += wsum[q];
      carry_s += t;
    }
    __syncthreads();
    if (threadIdx.x < 16) wsum[threadIdx.x] = 0;
    __syncthreads();
  }
  if (threadIdx.x == 0) ptr[w] = carry_s;
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ bucket,
                                                 int64_t nitems,
                                                 const int32_t* __restrict__ ptr,
                                                 int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nitems; i += stride) {
    const int b = bucket[i];
    const int pos = ptr[b] + atomicAdd(&cursor[b], 1);
    out[pos] = (int32_t)i;
  }
}

// The scatter with the same item ranges: each workgroup counts its items per
// bucket in LDS, takes one range of slots per non-empty bucket from the
// global cursor, and places its items there by LDS cursors.  The order inside
// a bucket depends on timing; the sort below makes it ascending.
__global__ __launch_bounds__(1024) void k_scatter_agg(const int32_t* __restrict__ bucket,
                                                      int64_t nitems, int w,
                                                      const int32_t* __restrict__ ptr,
                                                      int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ out) {
  __shared__ int32_t cur[kLdsBuckets];
  for (int b = threadIdx.x; b < w; b += blockDim.x) cur[b] = 0;
  __syncthreads();
  const int64_t per = (nitems + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < nitems ? i0 + per : nitems;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&cur[bucket[i]], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < w; b += blockDim.x) {
    const int c = cur[b];
    cur[b] = c ? ptr[b] + atomicAdd(&cursor[b], c) : 0;
  }
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int pos = atomicAdd(&cur[bucket[i]], 1);
    out[pos] = (int32_t)i;
  }
}

// Sort each bucket's items ascending (rank sort, one wave per bucket).  Items
// within a bucket are distinct, so rank = number of smaller items.  Reads the
// unsorted segments from `raw`, writes the sorted ones to `perm`.  A segment of
// up to kSortCap items is staged in LDS; a longer one (needs n*s/w > kSortCap on
// average) is placed kSortCap items per round, comparing against global memory.
constexpr int kSortCap = 2048;

__global__ __launch_bounds__(256) void k_bucket_sort(const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ raw,
                                                     int32_t* __restrict__ perm, int w) {
  __shared__ int32_t tile[4][kSortCap];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + wid;
  if (b >= w) return;
  const int beg = ptr[b], len = ptr[b + 1] - beg;
  if (len <= 0) return;
  if (len <= kSortCap) {
    for (int i = lane; i < len; i += 64) tile[wid][i] = raw[beg + i];
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < len; i += 64) {
      const int32_t e = tile[wid][i];
      int rank = 0;
      for (int q = 0; q < len; ++q) rank += tile[wid][q] < e;
      perm[beg + rank] = e;
    }
    return;
  }
  int32_t lo = -1;  // every item > lo is still to be placed
  int placed = 0;
  while (placed < len) {
    for (int i = lane; i < len; i += 64) {
      const int32_t e = raw[beg + i];
      if (e <= lo) continue;
      int rank = 0;
      for (int q = 0; q < len; ++q) {
        const int32_t f = raw[beg + q];
        rank += (f > lo) & (f < e);
      }
      if (rank < kSortCap) tile[wid][rank] = e;
    }
    __builtin_amdgcn_wave_barrier();
    const int took = (len - placed) < kSortCap ? (len - placed) : kSortCap;
    for (int i = lane; i < took; i += 64) perm[beg + placed + i] = tile[wid][i];
    lo = tile[wid][took - 1];
    __builtin_amdgcn_wave_barrier();
    placed += took;
  }
}

}  // namespace

void launch_hash(uint64_t seed, int64_t k, int s, int64_t n, int w, int32_t* bucket,
                 int8_t* sign, int32_t* count, hipStream_t st) {
  HashBases hb{};
  for (int r = 0; r < s && r < kMaxS; ++r)
    hb.base[r] = mix64(seed + kGolden * (1ull + (uint64_t)k * (uint64_t)s + (uint64_t)r));
  const int blk = w / s;
  if (count && w <= kLdsBuckets) {
    int64_t blocks = (n * s + 1023) / 1024;
    if (blocks > kAggBlocks) blocks = kAggBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_hash_agg, dim3((unsigned)blocks), dim3(1024), 0, st, hb, s, n, blk, w,
                       bucket, sign, count);
    return;
  }
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_hash, dim3((unsigned)blocks), dim3(256), 0, st, hb, s, n, blk, bucket,
                     sign, count);
}

void launch_bucket_scan(const int32_t* count, int32_t* ptr, int32_t* cursor, int w,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, count, ptr, cursor, w);
}

void launch_bucket_scatter(const int32_t* bucket, int64_t nitems, int w, const int32_t* ptr,
                           int32_t* cursor, int32_t* perm, hipStream_t st) {
  if (w <= kLdsBuckets) {
    int64_t blocks = (nitems + 1023) / 1024;
    if (blocks > kAggBlocks) blocks = kAggBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_scatter_agg, dim3((unsigned)blocks), dim3(1024), 0, st, bucket, nitems,
                       w, ptr, cursor, perm);
    return;
  }
  int64_t blocks = (nitems + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, st, bucket, nitems, ptr,
                     cursor, perm);
}

void launch_bucket_sort(const int32_t* ptr, const int32_t* raw, int32_t* perm, int w,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_bucket_sort, dim3((unsigned)((w + 3) / 4)), dim3(256), 0, st, ptr, raw,
                     perm, w);
}

}  // namespace skipm
