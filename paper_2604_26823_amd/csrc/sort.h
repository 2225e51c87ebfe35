// Stable least-significant-digit radix sort of (uint64 key, uint32 index)
// pairs, and the key transforms of rank-order matching (gfx950).
//
// Each pass sorts one 4-bit digit: a per-tile histogram, one exclusive scan
// of the digit-major histogram table, and a scatter in which every thread
// places a contiguous run of keys in input order, so equal digits keep their
// order across threads and tiles (stability is what makes ties rank by index).
#pragma once

#include "common.h"

namespace ic {
namespace sk {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;
constexpr int kDigits = 16;

// Order-preserving unsigned image of a float or double with -0 mapped to +0
// and larger values giving larger images.
__device__ __forceinline__ uint64_t ordered_bits(float v) {
  uint32_t b = __float_as_uint(v);
  if (b == 0x80000000u) b = 0;
  b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return b;
}
__device__ __forceinline__ uint64_t ordered_bits(double v) {
  uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
  if (b == 0x8000000000000000ull) b = 0;
  b = (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
  return b;
}
template <typename T>
__device__ __forceinline__ uint64_t descending_key(T v) {
  constexpr uint64_t mask = sizeof(T) == 4 ? 0xFFFFFFFFull : ~0ull;
  return (~ordered_bits(v)) & mask;
}

static __global__ __launch_bounds__(kThreads) void k_hist(const uint64_t* __restrict__ keys,
                                                   long long n, int shift,
                                                   uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t cnt[kDigits];
  if (threadIdx.x < kDigits) cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kTile;
  for (int i = threadIdx.x; i < kTile; i += kThreads) {
    const long long g = base + i;
    if (g < n) atomicAdd(&cnt[(keys[g] >> shift) & (kDigits - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kDigits) hist[(long long)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of n values in place, one block of 1024 threads.
static __global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* __restrict__ v, long long n) {
  __shared__ uint32_t part[1024];
  const long long per = (n + blockDim.x - 1) / blockDim.x;
  const long long lo = threadIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  uint32_t s = 0;
  for (long long i = lo; i < hi; ++i) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (long long i = lo; i < hi; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
}

static __global__ __launch_bounds__(kThreads) void k_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, long long n, int shift,
    const uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint64_t sk[kTile];
  __shared__ uint32_t sv[kTile];
  __shared__ uint32_t pre[kDigits * kThreads];
  __shared__ uint32_t wsum[kThreads];
  const long long base = (long long)blockIdx.x * kTile;
  for (int i = threadIdx.x; i < kTile; i += kThreads) {
    const long long g = base + i;
    sk[i] = g < n ? kin[g] : 0;
    sv[i] = g < n ? vin[g] : 0;
  }
  __syncthreads();
  const int t = threadIdx.x;
  uint32_t cnt[kDigits];
#pragma unroll
  for (int d = 0; d < kDigits; ++d) cnt[d] = 0;
  for (int i = 0; i < kItems; ++i) {
    const long long g = base + t * kItems + i;
    if (g < n) cnt[(sk[t * kItems + i] >> shift) & (kDigits - 1)]++;
  }
#pragma unroll
  for (int d = 0; d < kDigits; ++d) pre[d * kThreads + t] = cnt[d];
  __syncthreads();
  // exclusive scan over the digit-major table: thread t owns 16 consecutive entries
  uint32_t own[kDigits];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kDigits; ++j) {
    own[j] = pre[t * kDigits + j];
    s += own[j];
  }
  wsum[t] = s;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    uint32_t x = t >= off ? wsum[t - off] : 0;
    __syncthreads();
    wsum[t] += x;
    __syncthreads();
  }
  uint32_t run = wsum[t] - s;
#pragma unroll
  for (int j = 0; j < kDigits; ++j) {
    pre[t * kDigits + j] = run;
    run += own[j];
  }
  __syncthreads();
  uint32_t pos[kDigits];
#pragma unroll
  for (int d = 0; d < kDigits; ++d)
    pos[d] = hist[(long long)d * nblocks + blockIdx.x] + pre[d * kThreads + t] - pre[d * kThreads];
  for (int i = 0; i < kItems; ++i) {
    const long long g = base + t * kItems + i;
    if (g < n) {
      const uint64_t k = sk[t * kItems + i];
      const int d = (k >> shift) & (kDigits - 1);
      kout[pos[d]] = k;
      vout[pos[d]] = sv[t * kItems + i];
      pos[d]++;
    }
  }
}

template <typename T>
__global__ void k_desc_keys(const T* __restrict__ x, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ vals, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    keys[i] = descending_key<T>(x[i]);
    vals[i] = static_cast<uint32_t>(i);
  }
}

// keys[i] = small[vals[i]] (second-level key gathered through the order).
static __global__ void k_gather_u32_key(const uint32_t* __restrict__ small,
                                 const uint32_t* __restrict__ vals, uint64_t* __restrict__ keys,
                                 long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    keys[i] = small[vals[i]];
}

}  // namespace sk

// Sorts (keys, vals) ascending on the low nbits of keys, stably; the result
// ends in keys/vals (ka/va are scratch of the same size).  hist needs
// 16 * ceil(n / 4096) entries.
inline void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* ka, uint32_t* va,
                             uint32_t* hist, long long n, int nbits, hipStream_t st) {
  if (n <= 1) return;
  const int nblocks = static_cast<int>((n + sk::kTile - 1) / sk::kTile);
  uint64_t *kin = keys, *kout = ka;
  uint32_t *vin = vals, *vout = va;
  for (int shift = 0; shift < nbits; shift += 4) {
    sk::k_hist<<<nblocks, sk::kThreads, 0, st>>>(kin, n, shift, hist, nblocks);
    IC_LAUNCHED();
    sk::k_scan_excl<<<1, 1024, 0, st>>>(hist, (long long)sk::kDigits * nblocks);
    IC_LAUNCHED();
    sk::k_scatter<<<nblocks, sk::kThreads, 0, st>>>(kin, vin, kout, vout, n, shift, hist,
                                                   nblocks);
    IC_LAUNCHED();
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (kin != keys) {
    IC_HIP(hipMemcpyAsync(keys, kin, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    IC_HIP(hipMemcpyAsync(vals, vin, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  }
}

}  // namespace ic
