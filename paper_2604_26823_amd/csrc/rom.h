// Rank-order matching kernels (paper section 2.3.2): key construction for
// the real-space set (cells with R >= r_min) and for the Fourier-space k
// bins, target draws, and the scatter of sorted targets (gfx950).
#pragma once

#include "common.h"
#include "fields.h"
#include "sort.h"

namespace ic {
namespace rk {

// Real space: descending value key for every cell; second key 0 on the
// matched set (R >= r_min), 1 elsewhere, so the matched cells sort first.
template <typename T>
__global__ void k_real_keys(const T* __restrict__ s, const T* __restrict__ R, T r_min,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            uint32_t* __restrict__ second, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    keys[i] = sk::descending_key<T>(s[i]);
    vals[i] = static_cast<uint32_t>(i);
    second[i] = R[i] >= r_min ? 0u : 1u;
  }
}

// out[j] = src[idx[j]] for j < n.
template <typename T>
__global__ void k_gather(const T* __restrict__ src, const uint32_t* __restrict__ idx,
                         T* __restrict__ out, long long n) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x)
    out[j] = src[idx[j]];
}

// Targets of the real-space set and their descending keys: N(0,1) draw j.
template <typename T>
__global__ void k_real_targets(uint64_t event, uint64_t seed, T* __restrict__ tau,
                               uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                               long long n) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x) {
    const T v = static_cast<T>(fk::philox_draw(0, (uint64_t)j, 0, 2, event, seed));
    tau[j] = v;
    keys[j] = sk::descending_key<T>(v);
    vals[j] = static_cast<uint32_t>(j);
  }
}

// s[idx[j]] = tau[order[j]] for j < n: the j-th largest value gets the j-th
// largest target.
template <typename T>
__global__ void k_scatter_sorted(T* __restrict__ s, const uint32_t* __restrict__ idx,
                                 const T* __restrict__ tau, const uint32_t* __restrict__ order,
                                 long long n) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x)
    s[idx[j]] = tau[order[j]];
}

// Bin of half-spectrum mode f (kz, ky, kx its wave indices): the k bin of
// an independent mode with |k| >= k_min, else 255.
__device__ __forceinline__ uint32_t mode_bin(long long f, int n, double kf, double kmin,
                                             double dk, int nbins) {
  const int K = n / 2 + 1;
  const int kz = static_cast<int>(f % K);
  const long long r = f / K;
  const int ky = static_cast<int>(r % n), kx = static_cast<int>(r / n);
  bool independent = true;
  if (kz == 0 || kz == n / 2) {
    const int cx_ = (n - kx) & (n - 1), cy = (n - ky) & (n - 1);
    const long long conj = ((long long)cx_ * n + cy) * K + kz;
    independent = f < conj;
  }
  const int ix = kx < n / 2 ? kx : kx - n;
  const int iy = ky < n / 2 ? ky : ky - n;
  const double k = kf * sqrt((double)(ix * ix + iy * iy + kz * kz));
  if (!independent || k < kmin) return 255u;
  const int b = static_cast<int>(floor((k - kmin) / dk));
  return static_cast<uint32_t>(b < nbins - 1 ? b : nbins - 1);
}

// Fourier space: for every half-spectrum mode f = (kx n + ky)(n/2+1) + kz
// (stored at (kx n + ky) kp + kz), amplitude |z| = |Z_f| * scale, descending
// key, and second key = bin for matched modes (independent, |k| >= k_min)
// or 255.
template <typename T>
__global__ void k_mode_keys(const cx<T>* __restrict__ Z, int n, int kp, T scale, double kf,
                            double kmin,
                            double dk, int nbins, T* __restrict__ amp,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            uint32_t* __restrict__ second, long long H) {
  const int K = n / 2 + 1;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < H;
       f += (long long)gridDim.x * blockDim.x) {
    const int kz = static_cast<int>(f % K);
    const long long r = f / K;
    const cx<T> z = Z[r * kp + kz];
    const T a = sqrt(z.x * z.x + z.y * z.y) * scale;
    amp[f] = a;
    keys[f] = sk::descending_key<T>(a);
    vals[f] = static_cast<uint32_t>(f);
    second[f] = mode_bin(f, n, kf, kmin, dk, nbins);
  }
}

// Real/imaginary-part reading: element e = 2 f + c holds part c (0 = Re,
// 1 = Im) of mode f times scale, with its descending key and the bin of f
// as second key.
template <typename T>
__global__ void k_part_keys(const cx<T>* __restrict__ Z, int n, int kp, T scale, double kf,
                            double kmin, double dk, int nbins, T* __restrict__ val,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            uint32_t* __restrict__ second, long long H) {
  const int K = n / 2 + 1;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < H;
       f += (long long)gridDim.x * blockDim.x) {
    const int kz = static_cast<int>(f % K);
    const long long r = f / K;
    const cx<T> z = Z[r * kp + kz];
    const uint32_t bin = mode_bin(f, n, kf, kmin, dk, nbins);
    const T v[2] = {z.x * scale, z.y * scale};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const long long e = 2 * f + c;
      val[e] = v[c];
      keys[e] = sk::descending_key<T>(v[c]);
      vals[e] = static_cast<uint32_t>(e);
      second[e] = bin;
    }
  }
}

// End (last position + 1) of each bin's run in the bin-sorted keys, for
// bins < 255; entries of absent bins are left as they are (zero-filled by
// the caller).  The last element of a run is its only writer, so no atomics:
// a histogram by atomics serialises on the sorted input, where every lane of
// a wavefront hits the same counter.
static __global__ void k_bin_ends(const uint64_t* __restrict__ bins, uint32_t* __restrict__ ends,
                                  long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const uint64_t b = bins[i];
    if (b < 255 && (i + 1 == n || bins[i + 1] != b)) ends[b] = static_cast<uint32_t>(i + 1);
  }
}

// Target of sorted position i: bin b = bins[i], index within the bin
// j = i - start[b], draw kind (1 = Rayleigh, 0 = normal) of the given
// stream times mult; second key of the target sort is the bin.
template <typename T>
__global__ void k_fourier_targets(const uint64_t* __restrict__ bins,
                                  const uint32_t* __restrict__ start, int kind, uint64_t stream,
                                  double mult, uint64_t event,
                                  uint64_t seed, T* __restrict__ tau,
                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                  uint32_t* __restrict__ second, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const uint32_t b = static_cast<uint32_t>(bins[i]);
    const uint64_t j = (uint64_t)(i - start[b]);
    const T v = static_cast<T>(fk::philox_draw(kind, j, b, stream, event, seed) * mult);
    tau[i] = v;
    keys[i] = sk::descending_key<T>(v);
    vals[i] = static_cast<uint32_t>(i);
    second[i] = b;
  }
}

// Z_f <- tau * unscale * Z_f / |Z_f| (tau * unscale when Z_f = 0) for the
// matched mode f = idx[i], with the target tau[order[i]]; modes of the kz = 0
// and kz = n/2 planes also set their conjugate partner.
template <typename T>
__global__ void k_fourier_scatter(cx<T>* __restrict__ Z, int n, int kp,
                                  const uint32_t* __restrict__ idx,
                                  const T* __restrict__ tau, const uint32_t* __restrict__ order,
                                  T unscale, long long cnt) {
  const int K = n / 2 + 1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const long long f = idx[i];
    const T t = tau[order[i]] * unscale;
    const int kz = static_cast<int>(f % K);
    const long long r = f / K;
    const cx<T> z = Z[r * kp + kz];
    const T a = sqrt(z.x * z.x + z.y * z.y);
    const cx<T> v = a > T(0) ? mkc<T>(z.x * (t / a), z.y * (t / a)) : mkc<T>(t, T(0));
    Z[r * kp + kz] = v;
    if (kz == 0 || kz == n / 2) {
      const int ky = static_cast<int>(r % n), kx = static_cast<int>(r / n);
      const int cx_ = (n - kx) & (n - 1), cy = (n - ky) & (n - 1);
      Z[((long long)cx_ * n + cy) * kp + kz] = mkc<T>(v.x, -v.y);
    }
  }
}

// Real/imaginary-part reading: part c of mode f (element idx[i] = 2 f + c)
// <- tau[order[i]] * unscale.
template <typename T>
__global__ void k_part_scatter(cx<T>* __restrict__ Z, int n, int kp,
                               const uint32_t* __restrict__ idx, const T* __restrict__ tau,
                               const uint32_t* __restrict__ order, T unscale, long long cnt) {
  const int K = n / 2 + 1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const long long e = idx[i];
    const long long f = e >> 1;
    const int kz = static_cast<int>(f % K);
    T* z = reinterpret_cast<T*>(Z + (f / K) * kp + kz);
    z[e & 1] = tau[order[i]] * unscale;
  }
}

// After k_part_scatter: every matched mode of the kz = 0 and kz = n/2 planes
// (visited through its Re element) sets its conjugate partner.
template <typename T>
__global__ void k_part_mirror(cx<T>* __restrict__ Z, int n, int kp,
                              const uint32_t* __restrict__ idx, long long cnt) {
  const int K = n / 2 + 1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const long long e = idx[i];
    if (e & 1) continue;
    const long long f = e >> 1;
    const int kz = static_cast<int>(f % K);
    if (kz != 0 && kz != n / 2) continue;
    const long long r = f / K;
    const int ky = static_cast<int>(r % n), kx = static_cast<int>(r / n);
    const int cx_ = (n - kx) & (n - 1), cy = (n - ky) & (n - 1);
    const cx<T> v = Z[r * kp + kz];
    Z[((long long)cx_ * n + cy) * kp + kz] = mkc<T>(v.x, -v.y);
  }
}

}  // namespace rk
}  // namespace ic
