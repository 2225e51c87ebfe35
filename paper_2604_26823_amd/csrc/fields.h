// Grid-wise kernels: fills, 2LPT source and assembly, the observation model
// and loss with its adjoint seed, FP64 reductions, projection, L-BFGS
// vector updates and the counter-based generator (gfx950).
//
// Every reduction accumulates in FP64 and is deterministic: blocks write
// partial sums in a fixed order and one block adds them in a fixed order.
#pragma once

#include "common.h"

namespace ic {
namespace fk {

constexpr int kRedThreads = 256;

// Block-wide FP64 sum (blockDim.x == kRedThreads).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kRedThreads / 64; ++w) r += sh[w];
  }
  __syncthreads();
  return r;
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, T v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

// mu2 = phi_xx phi_yy + phi_xx phi_zz + phi_yy phi_zz - phi_xy^2 - phi_xz^2 - phi_yz^2
// (phi holds xx, yy, zz, xy, xz, yz, P apart).
template <typename T>
__global__ void k_mu2(const T* __restrict__ phi, T* __restrict__ mu, long long P) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < P;
       i += (long long)gridDim.x * blockDim.x) {
    const T xx = phi[i], yy = phi[P + i], zz = phi[2 * P + i];
    const T xy = phi[3 * P + i], xz = phi[4 * P + i], yz = phi[5 * P + i];
    mu[i] = xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz;
  }
}

// In place: phi <- phi_bar given mu2_bar (d mu2 / d phi_ii = sum of the other
// two diagonal terms, d mu2 / d phi_ij = -2 phi_ij).
template <typename T>
__global__ void k_phi_bar(T* __restrict__ phi, const T* __restrict__ mub, long long P) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < P;
       i += (long long)gridDim.x * blockDim.x) {
    const T m = mub[i];
    const T xx = phi[i], yy = phi[P + i], zz = phi[2 * P + i];
    phi[i] = m * (yy + zz);
    phi[P + i] = m * (xx + zz);
    phi[2 * P + i] = m * (xx + yy);
    phi[3 * P + i] *= T(-2) * m;
    phi[4 * P + i] *= T(-2) * m;
    phi[5 * P + i] *= T(-2) * m;
  }
}

// In place: d <- D1 Psi1 + D2 Psi2, p <- a^2 E (f1 D1 Psi1 + f2 D2 Psi2), with
// Psi1 held in d and Psi2 in p on entry ([3][P] each).
template <typename T>
__global__ void k_lpt_assemble(T* __restrict__ d, T* __restrict__ p, T cd1, T cd2, T cp1, T cp2,
                               long long n3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3;
       i += (long long)gridDim.x * blockDim.x) {
    const T psi1 = d[i], psi2 = p[i];
    d[i] = cd1 * psi1 + cd2 * psi2;
    p[i] = cp1 * psi1 + cp2 * psi2;
  }
}

// Observation model of the data grid (section 2.2.1, items 4-5).
template <typename T>
struct Obs {
  int poisson;           // 0: linear bias, Gaussian chi^2; 1: the paper's model
  T nbar, bias, r_min;   // bias: linear b (Gaussian model only)
  T alpha, delta_th, k;  // power-law index, sigmoid threshold and steepness
};

// Floor of 1 + delta in the power-law bias: the paper's rate vanishes in
// empty cells, where log lambda diverges; below the floor u is constant.
constexpr double kUFloor = 1e-6;

// Observation model and loss on the data grid.  delta = rho - 1 (one particle
// per data cell on average).  When R is given: lambda = nbar R (1 + b delta)
// (Gaussian model) or lambda = nbar R u^alpha sigmoid(K (delta - delta_th)),
// u = max(1 + delta, kUFloor) (Poisson model).  With counts also given, each
// masked cell (R >= r_min) adds to the data term D either (N - lambda)^2 /
// (nbar R), with adjoint seed 1/2 dD/d delta = b nbar R (lambda - N) /
// (nbar R), or -2 (N log lambda - lambda - log N!) (section 2.2.2), with seed
// (1 - N / lambda) dlambda/d delta.  Per-block FP64 partial sums of D, |s|^2
// and the masked-cell count go to part[3 * block + k].
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_loss(
    const T* __restrict__ rho, const int* __restrict__ counts, const T* __restrict__ R,
    const T* __restrict__ s, Obs<T> o, T* __restrict__ seed, T* __restrict__ delta_out,
    T* __restrict__ lambda_out, double* __restrict__ part, long long n,
    const T* __restrict__ zh, int lg) {
  __shared__ double sh[kRedThreads / 64];
  double chi = 0, ss = 0, cnt = 0;
  // kU cells per thread and round (grid stride apart), all their inputs
  // loaded before any is used and without a branch on the cell (indices
  // clamped, the halo value and the count selected rather than guarded), so
  // the loads of a round go out together.
  constexpr int kU = 4;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; i0 < n; i0 += kU * st) {
    T rv[kU], zv[kU], rr[kU], sv[kU];
    int nv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * st < n ? i0 + u * st : n - 1;
      // the data paint's z halo (layout [z / 8][x][y], grid side 2^lg)
      // completes the cells z = 0 mod 8
      zv[u] = zh ? zh[((i & ((1ll << lg) - 1)) >> 3 << (2 * lg)) | (i >> lg)] : T(0);
      rr[u] = R ? R[i] : T(0);
      nv[u] = counts ? counts[i] : 0;
      sv[u] = s ? s[i] : T(0);
      rv[u] = rho[i];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * st;
      if (i >= n) continue;
      const T rh = rv[u] + ((i & 7) == 0 ? zv[u] : T(0));
      const T delta = rh - T(1);
      const T r = rr[u];
      T sd = T(0);
      if (delta_out) delta_out[i] = delta;
      if (R) {
        T lam, dlam = T(0);
        if (o.poisson) {
          // u = 1 + delta is the painted density itself: taken from rho, not
          // from 1 + (rho - 1), whose cancellation would leave nearly empty
          // cells (u near the floor) with FP32 rounding of order 1e-7 / u
          const T uu = rh > T(kUFloor) ? rh : T(kUFloor);
          const T sig = T(1) / (T(1) + exp(-o.k * (delta - o.delta_th)));
          const T ua = pow(uu, o.alpha);
          lam = o.nbar * r * ua * sig;
          const T du = rh > T(kUFloor) ? o.alpha * ua / uu : T(0);
          dlam = o.nbar * r * (du * sig + ua * o.k * sig * (T(1) - sig));
        } else {
          lam = o.nbar * r * (T(1) + o.bias * delta);
        }
        if (lambda_out) lambda_out[i] = lam;
        if (counts && r >= o.r_min) {
          const int nc = nv[u];
          if (o.poisson) {
            const double l = static_cast<double>(lam), nn = static_cast<double>(nc);
            chi += 2.0 * (l - nn * log(l) + lgamma(nn + 1.0));
            sd = (T(1) - static_cast<T>(nc) / lam) * dlam;
          } else {
            const T var = o.nbar * r;
            const double res = static_cast<double>(nc) - static_cast<double>(lam);
            chi += res * res / static_cast<double>(var);
            sd = o.bias * o.nbar * r * (lam - static_cast<T>(nc)) / var;
          }
          cnt += 1.0;
        }
      }
      if (seed) seed[i] = sd;
      if (s) {
        const double v = static_cast<double>(sv[u]);
        ss += v * v;
      }
    }
  }
  chi = block_sum(chi, sh);
  ss = block_sum(ss, sh);
  cnt = block_sum(cnt, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = chi;
    part[3 * blockIdx.x + 1] = ss;
    part[3 * blockIdx.x + 2] = cnt;
  }
}

// out[k] = sum_b part[stride * b + k] for k < stride (one block; fixed order).
static __global__ __launch_bounds__(kRedThreads) void k_reduce_parts(const double* __restrict__ part,
                                                              int nblocks, int stride,
                                                              double* __restrict__ out) {
  __shared__ double sh[kRedThreads / 64];
  for (int k = 0; k < stride; ++k) {
    double v = 0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += part[stride * b + k];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[k] = v;
  }
}

// Largest |x| over n values: per-block maxima into part, then their
// maximum into out (one block).  Maxima do not depend on the order.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_absmax_parts(const T* __restrict__ x,
                                                              long long n,
                                                              double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64];
  double m = 0.0;
#pragma unroll 4  // several iterations' loads in flight; same summation order
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(static_cast<double>(x[i])));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRedThreads / 64; ++w) m = fmax(m, sh[w]);
    part[blockIdx.x] = fmax(m, sh[0]);
  }
}

static __global__ __launch_bounds__(kRedThreads) void k_max_parts(const double* __restrict__ part,
                                                                  int nblocks,
                                                                  double* __restrict__ out) {
  __shared__ double sh[kRedThreads / 64];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) m = fmax(m, part[b]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kRedThreads / 64; ++w) m = fmax(m, sh[w]);
    *out = m;
  }
}

// Partial sums of a . b (b may be null: sum of a) and of (a - shift)^2 with
// shift read from device memory (may be null).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot(const T* __restrict__ a,
                                                     const T* __restrict__ b,
                                                     double* __restrict__ part, long long n) {
  __shared__ double sh[kRedThreads / 64];
  double acc = 0;
#pragma unroll 4  // several iterations' loads in flight; same summation order
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double x = static_cast<double>(a[i]);
    acc += b ? x * static_cast<double>(b[i]) : x;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Partial sums of g . (a - b) with the difference taken in FP64.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot_diff(const T* __restrict__ g,
                                                          const T* __restrict__ a,
                                                          const T* __restrict__ b,
                                                          double* __restrict__ part,
                                                          long long n) {
  __shared__ double sh[kRedThreads / 64];
  double acc = 0;
#pragma unroll 4  // several iterations' loads in flight; same summation order
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += static_cast<double>(g[i]) * (static_cast<double>(a[i]) - static_cast<double>(b[i]));
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Partial sums of (x - mean)^2, mean = sum[0] / n read from device memory.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_centered_sq(const T* __restrict__ a,
                                                             const double* __restrict__ sum,
                                                             double* __restrict__ part,
                                                             long long n) {
  __shared__ double sh[kRedThreads / 64];
  const double mean = sum[0] / static_cast<double>(n);
  double acc = 0;
#pragma unroll 4  // several iterations' loads in flight; same summation order
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double x = static_cast<double>(a[i]) - mean;
    acc += x * x;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// y = a + alpha b (alpha FP64 on the host, applied in T); y may alias a or b.
template <typename T>
__global__ void k_axpy(const T* a, const T* b, T alpha, T* y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a[i] + alpha * b[i];
}

// One step of the L-BFGS two-loop recursion: y = s_in x + c X with
// c = cs (d[ia] - fb d[ib]) from FP64 scalars d left on the device by earlier
// reductions (ib < 0: no second term), then partial sums of V . y per block
// (V may be null).  y may alias x.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_lbfgs_update(
    const T* x, T s_in, const T* __restrict__ X, const double* __restrict__ d, int ia, int ib,
    double cs, double fb, T* y, const T* __restrict__ V, double* __restrict__ part, long long n) {
  __shared__ double sh[kRedThreads / 64];
  const T c = static_cast<T>(cs * (d[ia] - (ib >= 0 ? fb * d[ib] : 0.0)));
  double acc = 0;
  // kU elements per thread and round, loaded before any store (x may alias
  // y, so the compiler would not move later loads above a store itself);
  // the same elements in the same order as a plain grid-stride loop
  constexpr int kU = 4;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; i0 < n; i0 += kU * st) {
    T xv[kU], Xv[kU], Vv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * st < n ? i0 + u * st : n - 1;
      xv[u] = x[i];
      Xv[u] = X[i];
      Vv[u] = V ? V[i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * st;
      if (i >= n) continue;
      const T v = s_in * xv[u] + c * Xv[u];
      y[i] = v;
      if (V) acc += static_cast<double>(Vv[u]) * static_cast<double>(v);
    }
  }
  if (!V) return;
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// y = alpha x.
template <typename T>
__global__ void k_scale(const T* __restrict__ x, T alpha, T* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = alpha * x[i];
}

// y = a - b.
template <typename T>
__global__ void k_sub(const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ y,
                      long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

// ------------------------------------------------------------ Philox4x64-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two
// 64x64->128 multiplications with the Weyl key schedule.
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 r;
  r.v[0] = c0;
  r.v[1] = c1;
  r.v[2] = c2;
  r.v[3] = c3;
  return r;
}

__device__ __forceinline__ double unit_open(uint64_t w) {
  return (static_cast<double>(w >> 11) + 0.5) * 0x1.0p-53;
}

// kind 0: sqrt(-2 ln u0) cos(2 pi u1); kind 1: sqrt(-ln u0).
__device__ __forceinline__ double philox_draw(int kind, uint64_t j, uint64_t sub, uint64_t stream,
                                              uint64_t event, uint64_t seed) {
  U64x4 w = philox4x64_10(j, sub, stream, event, seed);
  const double u0 = unit_open(w.v[0]);
  if (kind == 1) return sqrt(-log(u0));
  const double u1 = unit_open(w.v[1]);
  return sqrt(-2.0 * log(u0)) * cospi(2.0 * u1);
}

template <typename T>
__global__ void k_philox(int kind, uint64_t sub, uint64_t stream, uint64_t event, uint64_t seed,
                         T* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = static_cast<T>(philox_draw(kind, (uint64_t)i, sub, stream, event, seed));
}

// White-noise upsampling (section 3, the resolution schedule): the modes of
// a coarse field with every wave index strictly inside (-nl/2, nl/2) replace
// those of a fine spectrum, times scale = (nh/nl)^{3/2} (the unnormalised DFT
// of unit white noise grows as the cell count).  lo: dense coarse half
// spectrum [nl][nl][nl/2+1]; hi: stored fine half spectrum [nh][nh][kp].  One
// thread per coarse (i, j, kz < nl/2); the coarse Nyquist rows are skipped.
template <typename T>
__global__ void k_embed_coarse(const cx<T>* __restrict__ lo, int nl, cx<T>* __restrict__ hi,
                               int nh, int kp, T scale) {
  const int h = nl / 2;
  const long long total = (long long)nl * nl * h;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int kz = static_cast<int>(t % h);
    const long long r = t / h;
    const int j = static_cast<int>(r % nl);
    const int i = static_cast<int>(r / nl);
    if (i == h || j == h) continue;
    const int fi = i < h ? i : i + (nh - nl);
    const int fj = j < h ? j : j + (nh - nl);
    const cx<T> v = lo[((long long)i * nl + j) * (h + 1) + kz];
    hi[((long long)fi * nh + fj) * kp + kz] = cscale<T>(v, scale);
  }
}

// One projection pass: out = (x - mean) / std with mean = sum[0]/n and
// std = sqrt(sq[0]/n); |out| > s_th is replaced by the reset draw of that
// element (counter sub word = sub).  The reset count goes to part[block].
// x may equal out.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_project(
    const T* x, const double* __restrict__ sum, const double* __restrict__ sq, T s_th,
    uint64_t sub, uint64_t event, uint64_t seed, T* out, double* __restrict__ part,
    long long n) {
  __shared__ double sh[kRedThreads / 64];
  const double mean = sum[0] / static_cast<double>(n);
  const double sd = sqrt(sq[0] / static_cast<double>(n));
  double resets = 0;
  // four elements per thread and round, loaded before any store (x may be
  // out); the same elements in the same order as a plain grid-stride loop
  constexpr int kU = 4;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x; i0 < n; i0 += kU * st) {
    T xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) xv[u] = x[i0 + u * st < n ? i0 + u * st : n - 1];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * st;
      if (i >= n) continue;
      T z = static_cast<T>((static_cast<double>(xv[u]) - mean) / sd);
      if (fabs(z) > s_th) {
        z = static_cast<T>(philox_draw(0, (uint64_t)i, sub, 1, event, seed));
        resets += 1.0;
      }
      out[i] = z;
    }
  }
  resets = block_sum(resets, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = resets;
}

// Non-finite check: part[block] = count of non-finite values.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_count_nonfinite(const T* __restrict__ x,
                                                                 double* __restrict__ part,
                                                                 long long n) {
  __shared__ double sh[kRedThreads / 64];
  double bad = 0;
#pragma unroll 4  // several iterations' loads in flight; same summation order
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad += 1.0;
  bad = block_sum(bad, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = bad;
}

}  // namespace fk
}  // namespace ic
