// Stockham FFT passes staged in LDS for gfx950 (64-wide wavefronts).
//
// Each 1D transform of length n is done by n / R_max threads ("lanes") that
// hold R_max points in registers; a stage is one radix-R butterfly per
// (lane, batch) with the Stockham autosort index map, so data stays in
// natural order and every stage reads contiguous element runs.  Stages
// exchange data through LDS; the first stage reads global memory and the
// last one writes it, so each pass touches HBM once per element in and out.
//
// Strided passes (y, x) put consecutive lines of the batch on consecutive
// threads, so every global access of a wavefront covers LINES consecutive
// complex values (128 B in FP32); the z pass keeps lanes of one line on
// consecutive threads because its lines are contiguous.
#pragma once

#include <type_traits>

#include "fft.h"

namespace ic {
namespace fftk {

// Radix plan (up to three stages) for complex length n.
template <int n> struct Plan;
#define IC_FFT_PLAN(N, A, B, C)                                 \
  template <> struct Plan<N> {                                  \
    static constexpr int R0 = A, R1 = B, R2 = C;                \
    static constexpr int S = (B == 1) ? 1 : ((C == 1) ? 2 : 3); \
    static constexpr int RMAX = (A > B ? (A > C ? A : C) : (B > C ? B : C)); \
    static constexpr int TPL = N / RMAX;                        \
  };
IC_FFT_PLAN(2, 2, 1, 1)
IC_FFT_PLAN(4, 4, 1, 1)
IC_FFT_PLAN(8, 8, 1, 1)
IC_FFT_PLAN(16, 16, 1, 1)
IC_FFT_PLAN(32, 8, 4, 1)
IC_FFT_PLAN(64, 8, 8, 1)
IC_FFT_PLAN(128, 16, 8, 1)
IC_FFT_PLAN(256, 16, 16, 1)
IC_FFT_PLAN(512, 8, 8, 8)
IC_FFT_PLAN(1024, 16, 8, 8)
#undef IC_FFT_PLAN

// Radix plans of the fused x passes, which hold a line's spectrum in
// registers across several transforms: PlanX for the scatter (one forward,
// several inverses), PlanG for the gather (several forwards, one inverse);
// both default to Plan<n>.  The gather at n = 256 takes radix 8 first, so a
// thread holds 8 values instead of 16 and more waves fit per SIMD.
template <int n> struct PlanX : Plan<n> {};
template <int n> struct PlanG : Plan<n> {};
template <> struct PlanG<256> {
  static constexpr int R0 = 8, R1 = 8, R2 = 4;
  static constexpr int S = 3;
  static constexpr int RMAX = 8;
  static constexpr int TPL = 256 / RMAX;
};

// cos and sin of 2 pi m / 16, m = 0..7.
__device__ constexpr double kC16[8] = {1.0,
                                       0.92387953251128675613,
                                       0.70710678118654752440,
                                       0.38268343236508977173,
                                       0.0,
                                       -0.38268343236508977173,
                                       -0.70710678118654752440,
                                       -0.92387953251128675613};
__device__ constexpr double kS16[8] = {0.0,
                                       0.38268343236508977173,
                                       0.70710678118654752440,
                                       0.92387953251128675613,
                                       1.0,
                                       0.92387953251128675613,
                                       0.70710678118654752440,
                                       0.38268343236508977173};

// x * exp(-+ 2 pi i k / R) (forward: minus), k < R/2.
template <typename T, int R, bool FWD>
__device__ __forceinline__ cx<T> rot(cx<T> x, int k) {
  if (k == 0) return x;
  if (4 * k == R) return FWD ? mkc<T>(x.y, -x.x) : mkc<T>(-x.y, x.x);
  const int m = k * (16 / R);
  const T c = static_cast<T>(kC16[m]);
  const T s = FWD ? -static_cast<T>(kS16[m]) : static_cast<T>(kS16[m]);
  return mkc<T>(x.x * c - x.y * s, x.x * s + x.y * c);
}

// In-register DFT of length R (R a power of two <= 16), decimation in time.
template <typename T, int R, bool FWD>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    cx<T> a = v[0];
    v[0] = cadd<T>(a, v[1]);
    v[1] = csub<T>(a, v[1]);
  } else {
    cx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<T, R / 2, FWD>(e);
    dft<T, R / 2, FWD>(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      cx<T> t = rot<T, R, FWD>(o[k], k);
      v[k] = cadd<T>(e[k], t);
      v[k + R / 2] = csub<T>(e[k], t);
    }
  }
}

// One Stockham stage of radix R on a length-n transform whose sub-transforms
// have size Ns.  Butterfly j reads elements j + r n/R, twiddles them by
// W_{Ns R}^{(j mod Ns) r} and writes (j - j mod Ns) R + j mod Ns + r Ns.
// tw is the table exp(-2 pi i m / (n * tws)).  All reads of the stage
// happen before the (optional) barrier and all writes after it, so a stage
// may write the buffer it read.
template <typename T, int n, int R, int TPL, bool FWD, class Load, class Store>
__device__ __forceinline__ void stage(int lane, int Ns, const cx<T>* __restrict__ tw, int tws,
                                      Load&& load, Store&& store, bool sync_before_store) {
  constexpr int NB = n / R;
  static_assert(NB % TPL == 0, "butterflies must divide evenly over lanes");
  constexpr int BPT = NB / TPL;
  cx<T> v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jb = lane + b * TPL;
    const int k = jb & (Ns - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = load(jb + r * NB);
    if (Ns > 1) {
      const int step = (n / (Ns * R)) * k;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = tw[step * r * tws];
        if (!FWD) w.y = -w.y;
        v[b][r] = cmul<T>(v[b][r], w);
      }
    }
    dft<T, R, FWD>(v[b]);
  }
  if (sync_before_store) __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jb = lane + b * TPL;
    const int k = jb & (Ns - 1);
    const int base = (jb - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) store(base + r * Ns, v[b][r]);
  }
}

// Full length-n transform: first stage from load0, intermediate stages in
// the LDS buffer buf (element e of this thread's line at buf[lidx(e)]), last
// stage to storeL.
template <typename T, int n, bool FWD, class Load, class Store, class LIdx>
__device__ __forceinline__ void fft_line(int lane, cx<T>* buf, LIdx lidx,
                                         const cx<T>* __restrict__ tw, int tws, Load&& load0,
                                         Store&& storeL) {
  using P = Plan<n>;
  constexpr int TPL = P::TPL;
  auto ld = [&](int e) { return buf[lidx(e)]; };
  auto st = [&](int e, cx<T> v) { buf[lidx(e)] = v; };
  if constexpr (P::S == 1) {
    stage<T, n, P::R0, TPL, FWD>(lane, 1, tw, tws, load0, storeL, true);
  } else if constexpr (P::S == 2) {
    stage<T, n, P::R0, TPL, FWD>(lane, 1, tw, tws, load0, st, true);
    __syncthreads();
    stage<T, n, P::R1, TPL, FWD>(lane, P::R0, tw, tws, ld, storeL, true);
  } else {
    stage<T, n, P::R0, TPL, FWD>(lane, 1, tw, tws, load0, st, true);
    __syncthreads();
    stage<T, n, P::R1, TPL, FWD>(lane, P::R0, tw, tws, ld, st, true);
    __syncthreads();
    stage<T, n, P::R2, TPL, FWD>(lane, P::R0 * P::R1, tw, tws, ld, storeL, true);
  }
}

// Transforms that keep the last stage in registers.  The last stage of a
// Stockham plan writes element jb + r n / R_last from butterfly jb, and the
// first stage (sub-size 1) of a plan that starts with radix R_last reads
// exactly those elements into butterfly jb.  So a forward transform can end
// in registers and an inverse transform in the reversed radix order can
// start from them, with no LDS round trip in between: the fused x passes
// hold a line's spectrum in registers while it is multiplied (and summed),
// and need one LDS tile instead of two.
template <int n, class PL = PlanX<n>>
struct XPlan {
  using P = PL;
  static constexpr int S = P::S;
  static constexpr int RL = S == 1 ? P::R0 : (S == 2 ? P::R1 : P::R2);  // last forward radix
  static constexpr int Q1 = S == 1 ? 1 : (S == 2 ? P::R0 : P::R1);      // inverse radices
  static constexpr int Q2 = S == 3 ? P::R0 : 1;                         // after RL
  static constexpr int TPL = P::TPL;
  static constexpr int NBL = n / RL;
  static constexpr int BPT = NBL / TPL;
};

// A stage whose outputs stay in registers: v[b][r] holds element
// lane + b TPL + r n / R (valid as the last stage, sub-size n / R).
template <typename T, int n, int R, int TPL, bool FWD, class Load>
__device__ __forceinline__ void stage_to_regs(int lane, int Ns, const cx<T>* __restrict__ tw,
                                              Load&& load, cx<T> (&v)[n / R / TPL][R]) {
  constexpr int NB = n / R;
  constexpr int BPT = NB / TPL;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jb = lane + b * TPL;
    const int k = jb & (Ns - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = load(jb + r * NB);
    if (Ns > 1) {
      const int step = (n / (Ns * R)) * k;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = tw[step * r];
        if (!FWD) w.y = -w.y;
        v[b][r] = cmul<T>(v[b][r], w);
      }
    }
    dft<T, R, FWD>(v[b]);
  }
}

// A first stage (sub-size 1) from registers: butterfly jb = lane + b TPL
// takes v[b][r] as its element jb + r n / R and stores element jb R + r.
// With sync, a barrier precedes the stores (earlier readers of the LDS
// tile are done).
template <typename T, int n, int R, int TPL, bool FWD, class Store>
__device__ __forceinline__ void stage_from_regs(int lane, cx<T> (&v)[n / R / TPL][R],
                                                Store&& store, bool sync) {
  constexpr int BPT = n / R / TPL;
#pragma unroll
  for (int b = 0; b < BPT; ++b) dft<T, R, FWD>(v[b]);
  if (sync) __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jb = lane + b * TPL;
#pragma unroll
    for (int r = 0; r < R; ++r) store(jb * R + r, v[b][r]);
  }
}

// Forward length-n transform from load0 ending in registers (XPlan layout);
// the first store into buf follows a barrier.
template <typename T, int n, class PL, class Load, class LIdx>
__device__ __forceinline__ void fft_fwd_to_regs(int lane, cx<T>* buf, LIdx lidx,
                                                const cx<T>* __restrict__ tw, Load&& load0,
                                                cx<T> (&v)[XPlan<n, PL>::BPT][XPlan<n, PL>::RL]) {
  using P = PL;
  constexpr int TPL = P::TPL;
  auto ld = [&](int e) { return buf[lidx(e)]; };
  auto st = [&](int e, cx<T> x) { buf[lidx(e)] = x; };
  if constexpr (P::S == 1) {
    stage_to_regs<T, n, P::R0, TPL, true>(lane, 1, tw, load0, v);
  } else if constexpr (P::S == 2) {
    stage<T, n, P::R0, TPL, true>(lane, 1, tw, 1, load0, st, true);
    __syncthreads();
    stage_to_regs<T, n, P::R1, TPL, true>(lane, P::R0, tw, ld, v);
  } else {
    stage<T, n, P::R0, TPL, true>(lane, 1, tw, 1, load0, st, true);
    __syncthreads();
    stage<T, n, P::R1, TPL, true>(lane, P::R0, tw, 1, ld, st, true);
    __syncthreads();
    stage_to_regs<T, n, P::R2, TPL, true>(lane, P::R0 * P::R1, tw, ld, v);
  }
}

// Inverse length-n transform starting from registers in the XPlan layout,
// radices in the reversed order, last stage to storeL; the first store into
// buf follows a barrier.  v is consumed.
template <typename T, int n, class PL, class Store, class LIdx>
__device__ __forceinline__ void fft_inv_from_regs(int lane, cx<T>* buf, LIdx lidx,
                                                  const cx<T>* __restrict__ tw,
                                                  cx<T> (&v)[XPlan<n, PL>::BPT][XPlan<n, PL>::RL],
                                                  Store&& storeL) {
  using X = XPlan<n, PL>;
  constexpr int TPL = X::TPL;
  auto ld = [&](int e) { return buf[lidx(e)]; };
  auto st = [&](int e, cx<T> x) { buf[lidx(e)] = x; };
  if constexpr (X::S == 1) {
    stage_from_regs<T, n, X::RL, TPL, false>(lane, v, storeL, false);
  } else if constexpr (X::S == 2) {
    stage_from_regs<T, n, X::RL, TPL, false>(lane, v, st, true);
    __syncthreads();
    stage<T, n, X::Q1, TPL, false>(lane, X::RL, tw, 1, ld, storeL, true);
  } else {
    stage_from_regs<T, n, X::RL, TPL, false>(lane, v, st, true);
    __syncthreads();
    stage<T, n, X::Q1, TPL, false>(lane, X::RL, tw, 1, ld, st, true);
    __syncthreads();
    stage<T, n, X::Q2, TPL, false>(lane, X::RL * X::Q1, tw, 1, ld, storeL, true);
  }
}

// ---------------------------------------------------------------- sizing
template <typename T, int N> struct ZCfg {
  static constexpr int n = N / 2;
  static constexpr int TPL = Plan<n>::TPL;
  static constexpr int LINES0 = 256 / TPL;
  static constexpr int LINES = LINES0 > 64 ? 64 : (LINES0 < 1 ? 1 : LINES0);
  static constexpr int THREADS = LINES * TPL;
  // LDS line stride (complex): one pad element per 16 (zl) plus two, so
  // the stride-16 accesses of the radix-16 stage fall in different banks.
  static constexpr int LS = n + n / 16 + 2;
};

// Padded LDS position of element e of a z line.
__device__ __forceinline__ int zl(int e) { return e + (e >> 4); }

template <typename T, int N> struct SCfg {  // strided C2C passes
  static constexpr int TPL = Plan<N>::TPL;
  static constexpr int LINES0 = sizeof(T) == 4 ? 16 : (N >= 1024 ? 4 : 8);
  static constexpr int LINES = (N <= 16) ? 64 : LINES0;
  static constexpr int THREADS = LINES * TPL;
  static constexpr int LP = LINES + 1;  // padded LDS element stride
};

template <typename T, int N, class PL = PlanX<N>> struct FCfg {  // fused x passes
  static constexpr int TPL = PL::TPL;
  // waves per SIMD the register allocation must allow: the FP32 scatter
  // otherwise takes just over half the register file (one wave per SIMD)
  static constexpr int MINW = (sizeof(T) == 4 && N <= 512) ? 2 : 1;
  static constexpr int LINES = (N <= 16) ? 64
                               : (sizeof(T) == 4 ? (N <= 512 ? 16 : 8)
                                                 : (N <= 512 ? 8 : 2));
  static constexpr int THREADS = LINES * TPL;
  static constexpr int LP = LINES + 1;
};

template <typename T>
__device__ __forceinline__ void load_table(cx<T>* dst, const cx<T>* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------ z pass R2C
// Element e of z row `line` (its complex pair 2e, 2e + 1) of
// alpha (a + zh) + beta b, without a branch: ZH and B are compile-time, and
// the z-halo value (added to the cells z = 0 mod 8) is loaded for every e and
// selected, so the loads of a transform's first stage are all issued before
// its first wait (a branch per element made each load wait for the previous).
template <typename T, int N, bool ZH, bool B>
__device__ __forceinline__ cx<T> r2c_elem(const cx<T>* __restrict__ ain,
                                          const cx<T>* __restrict__ bin,
                                          const T* __restrict__ zh, size_t line, int e,
                                          T alpha, T beta) {
  cx<T> u = ain[e];
  if constexpr (ZH) {
    const T z = zh[(size_t)(2 * e / kZHalo) * N * N + line];
    u.x += (e & (kZHalo / 2 - 1)) == 0 ? z : static_cast<T>(0);
  }
  cx<T> v = cscale<T>(u, alpha);
  if constexpr (B) {
    const cx<T> w = bin[e];
    v.x += beta * w.x;
    v.y += beta * w.y;
  }
  return v;
}

// zh (nullable): a paint's z halo, one value per eight cells along z, added
// to the cells z = 0 mod 8 of a (the value of cell z of line L = x N + y is
// zh[(z / 8) N^2 + L]).
template <typename T, int N, bool ZH, bool B>
__global__ __launch_bounds__((ZCfg<T, N>::THREADS)) void k_r2c_z(
    const T* __restrict__ a, T alpha, const T* __restrict__ b, T beta,
    cx<T>* __restrict__ out, const cx<T>* __restrict__ twg, int nlines, int kp,
    const T* __restrict__ zh) {
  using C = ZCfg<T, N>;
  constexpr int n = C::n;
  __shared__ cx<T> buf[C::LINES * C::LS];
  __shared__ cx<T> tw[N];
  load_table<T>(tw, twg, N);  // visible after the first stage's barrier, before any use
  const int lane = threadIdx.x % C::TPL;
  const int l = threadIdx.x / C::TPL;
  const int line = blockIdx.x * C::LINES + l;
  const bool valid = line < nlines;
  // past the last line: row 0 is transformed and not stored
  const size_t lrow = valid ? static_cast<size_t>(line) : 0;
  const cx<T>* ain = reinterpret_cast<const cx<T>*>(a + lrow * N);
  const cx<T>* bin = B ? reinterpret_cast<const cx<T>*>(b + lrow * N) : nullptr;
  auto load0 = [&](int e) -> cx<T> {
    return r2c_elem<T, N, ZH, B>(ain, bin, zh, lrow, e, alpha, beta);
  };
  cx<T>* lb = buf + l * C::LS;
  auto lidx = [&](int e) { return l * C::LS + zl(e); };
  auto storeL = [&](int e, cx<T> v) { lb[zl(e)] = v; };
  fft_line<T, n, true>(lane, buf, lidx, tw, 2, load0, storeL);
  __syncthreads();
  if (!valid) return;
  cx<T>* o = out + (size_t)line * kp;
  const T half = static_cast<T>(0.5);
  for (int k = lane; k <= n; k += C::TPL) {
    cx<T> zk = lb[zl(k == n ? 0 : k)];
    cx<T> zc = cconj<T>(lb[zl(k == 0 ? 0 : n - k)]);
    cx<T> e = cscale<T>(cadd<T>(zk, zc), half);
    cx<T> d = cscale<T>(csub<T>(zk, zc), half);
    // X[k] = E + W^k (-i D), W = exp(-2 pi i / N)
    cx<T> mid = mkc<T>(d.y, -d.x);
    o[k] = cadd<T>(e, cmul<T>(tw[k], mid));
  }
}

// ------------------------------------------------------------ z pass C2R
template <typename T, int N>
__global__ __launch_bounds__((ZCfg<T, N>::THREADS)) void k_c2r_z(
    const cx<T>* __restrict__ in, T* __restrict__ out, T alpha, const T* __restrict__ aux,
    T beta, const cx<T>* __restrict__ twg, int nlines, int kp) {
  using C = ZCfg<T, N>;
  constexpr int n = C::n;
  __shared__ cx<T> buf[C::LINES * C::LS];
  __shared__ cx<T> tw[N];
  load_table<T>(tw, twg, N);
  const int lane = threadIdx.x % C::TPL;
  const int l = threadIdx.x / C::TPL;
  const int line = blockIdx.x * C::LINES + l;
  const bool valid = line < nlines;
  cx<T>* lb = buf + l * C::LS;
  // the row's n + 1 values, all loads out before the first wait (no branch:
  // indices clamped, lines past the end read line 0 and store zeros)
  const cx<T>* src = in + (valid ? (size_t)line : 0) * kp;
  constexpr int KS = n / C::TPL + 1;
  cx<T> rv[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) rv[j] = src[min(lane + j * C::TPL, n)];
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    const int k = lane + j * C::TPL;
    if (k > n) continue;
    cx<T> v = valid ? rv[j] : mkc<T>(0, 0);
    if (k == 0 || k == n) v.y = 0;  // the real transform ignores these imaginary parts
    lb[zl(k)] = v;
  }
  __syncthreads();
  auto load0 = [&](int e) -> cx<T> {
    cx<T> xk = lb[zl(e)];
    cx<T> xc = cconj<T>(lb[zl(n - e)]);
    cx<T> s = cadd<T>(xk, xc);
    cx<T> d = csub<T>(xk, xc);
    cx<T> w = cconj<T>(tw[e]);  // exp(+2 pi i e / N)
    cx<T> wd = cmul<T>(w, d);
    return mkc<T>(s.x - wd.y, s.y + wd.x);  // s + i w d
  };
  auto lidx = [&](int e) { return l * C::LS + zl(e); };
  cx<T>* dst = reinterpret_cast<cx<T>*>(out + (size_t)line * N);
  const cx<T>* ax = aux ? reinterpret_cast<const cx<T>*>(aux + (size_t)line * N) : nullptr;
  auto storeL = [&](int e, cx<T> v) {
    if (!valid) return;
    cx<T> r = cscale<T>(v, alpha);
    if (ax) {
      cx<T> u = ax[e];
      r.x += beta * u.x;
      r.y += beta * u.y;
    }
    dst[e] = r;
  };
  fft_line<T, n, false>(lane, buf, lidx, tw, 2, load0, storeL);
}

// ------------------------------------------ fused z and y passes (FP32, n = 256)
// One workgroup transforms a whole x plane along z and y, so the plane's half
// spectrum crosses HBM once instead of three times.  The plane (256 rows y of
// 129 values kz) does not fit in LDS, so two identities shrink it:
//  * the columns kz = 0 and kz = n/2 are real along y (the z transform of a
//    real row is real there), so they travel as one complex column
//    c(y) = X(y, 0) + i X(y, n/2): 128 complex columns;
//  * one radix-2 step of the length-256 y transform splits it into two
//    length-128 transforms: the even outputs are the transform of
//    u(y) + u(y + 128), the odd ones that of (u(y) - u(y + 128)) W^y.
// A 128 x 128 LDS tile plus 16 values per thread in registers then hold the
// plane.  Forward: z transforms of rows 0-127 (through the tile, into
// registers), of rows 128-255 (into the tile); the radix-2 step (sums to the
// tile, differences to registers); the 128 even-output column transforms,
// then the odd ones; the packed column's outputs are separated last
// (X0 = (C[k] + conj C[-k]) / 2, X_{n/2} = (C[k] - conj C[-k]) / 2i).  The
// inverse mirrors it; its packed column needs the kz = 0 and n/2 columns to
// be Hermitian along y, which holds for the spectrum of any real field and
// for the k-space multipliers applied to one (even ones real, odd ones
// imaginary, the derivative ones zero at the Nyquist index).
template <typename T, int N>
struct ZYCfg {
  static constexpr bool ok = false;
};
template <>
struct ZYCfg<float, 256> {
  static constexpr bool ok = true;
  static constexpr int n = 128;                  // z row (complex), tile rows and columns
  static constexpr int TPL = Plan<n>::TPL;       // threads per row or column transform
  static constexpr int THREADS = n * TPL;        // 1024
  static constexpr int LS = n + n / 16 + 2;      // tile row stride, as the z pass
  static constexpr int OWN = THREADS / n;        // thread t owns rows t / n + OWN j of column t % n
  static constexpr int PER = n / OWN;            // 16 held values per thread
};

template <typename T, int N, bool ZH, bool B>
__global__ __launch_bounds__((ZYCfg<T, N>::THREADS)) void k_r2c_zy(
    const T* __restrict__ a, T alpha, const T* __restrict__ b, T beta,
    cx<T>* __restrict__ out, const cx<T>* __restrict__ twg, int kp,
    const T* __restrict__ zh) {
  using C = ZYCfg<T, N>;
  constexpr int n = C::n;
  __shared__ cx<T> buf[n * C::LS];
  __shared__ cx<T> tw[N];
  __shared__ cx<T> pk[2 * n];  // the packed column's even and odd outputs
  load_table<T>(tw, twg, N);  // visible after the first stage's barrier, before any use
  const int t = threadIdx.x;
  const size_t x = blockIdx.x;
  const int lane = t % C::TPL, l = t / C::TPL;  // z phase: lane of tile row l
  const int c = t % n, r0 = t / n;              // column phase and held values
  const T half = static_cast<T>(0.5);
  // held values: PER - SPARE in registers, the rest in LDS (the register
  // file is full)
  constexpr int SPARE = 1;
  __shared__ cx<T> spare[SPARE * C::THREADS];
  cx<T> keep[C::PER - SPARE];
  auto held = [&](int j) -> cx<T>& {
    return j < C::PER - SPARE ? keep[j] : spare[(j - (C::PER - SPARE)) * C::THREADS + t];
  };
  cx<T>* lb = buf + l * C::LS;
  // the half's z-halo values, staged in the tile as [z / 8][row] by coalesced
  // loads (a row's 32 values lie a plane apart in zh)
  constexpr int NZ = N / kZHalo;
  static_assert(NZ * C::n % C::THREADS == 0, "z-halo staging: whole rounds");
  const T* zt = reinterpret_cast<const T*>(buf);
  for (int h = 0; h < 2; ++h) {
    const size_t line = x * N + h * n + l;
    const cx<T>* ain = reinterpret_cast<const cx<T>*>(a + line * N);
    const cx<T>* bin = B ? reinterpret_cast<const cx<T>*>(b + line * N) : nullptr;
    if constexpr (ZH) {
      if (h == 1) __syncthreads();  // the first half's held values are read
      T* zw = reinterpret_cast<T*>(buf);
      constexpr int QZ = NZ * n / C::THREADS;
      T zv[QZ];
#pragma unroll
      for (int q = 0; q < QZ; ++q) {
        const int i = t + q * C::THREADS;
        zv[q] = zh[(size_t)(i / n) * N * N + x * N + h * n + i % n];
      }
#pragma unroll
      for (int q = 0; q < QZ; ++q) zw[t + q * C::THREADS] = zv[q];
      __syncthreads();
    }
    auto load0 = [&](int e) -> cx<T> {  // no branch: all loads out before the first wait
      cx<T> u = ain[e];
      if constexpr (ZH) {
        const T z = zt[(2 * e / kZHalo) * n + l];
        u.x += (e & (kZHalo / 2 - 1)) == 0 ? z : static_cast<T>(0);
      }
      cx<T> v = cscale<T>(u, alpha);
      if constexpr (B) {
        const cx<T> w = bin[e];
        v.x += beta * w.x;
        v.y += beta * w.y;
      }
      return v;
    };
    auto lidx = [&](int e) { return l * C::LS + zl(e); };
    auto storeL = [&](int e, cx<T> v) { lb[zl(e)] = v; };
    fft_line<T, n, true>(lane, buf, lidx, tw, 2, load0, storeL);
    __syncthreads();
    // the real transform's split, in place, pair (k, n - k) by one thread:
    // X[k] = E + W^k (-i D), E, D = (Z[k] +- conj Z[n - k]) / 2; X[0] and
    // X[n] (both real) packed into slot 0
    for (int k = lane; k <= n / 2; k += C::TPL) {
      const cx<T> zk = lb[zl(k)];
      if (k == 0) {
        lb[zl(0)] = mkc<T>(zk.x + zk.y, zk.x - zk.y);
        continue;
      }
      const cx<T> zm = lb[zl(n - k)];
      auto split = [&](cx<T> p, cx<T> q, int j) {
        const cx<T> qc = cconj<T>(q);
        const cx<T> e = cscale<T>(cadd<T>(p, qc), half);
        const cx<T> d = cscale<T>(csub<T>(p, qc), half);
        return cadd<T>(e, cmul<T>(tw[j], mkc<T>(d.y, -d.x)));
      };
      lb[zl(k)] = split(zk, zm, k);
      if (k != n / 2) lb[zl(n - k)] = split(zm, zk, n - k);
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int j = 0; j < C::PER; ++j) held(j) = buf[(r0 + C::OWN * j) * C::LS + zl(c)];
    }
    // the second half's first tile store follows a barrier in fft_line
  }
  // radix-2 step along y: rows y (held) and y + n (tile)
#pragma unroll
  for (int j = 0; j < C::PER; ++j) {
    const int y = r0 + C::OWN * j;
    cx<T>* q = buf + y * C::LS + zl(c);
    const cx<T> lo = held(j), hi = *q;
    *q = cadd<T>(lo, hi);
    held(j) = cmul<T>(csub<T>(lo, hi), tw[y]);
  }
  __syncthreads();
  auto cidx = [&](int e) { return e * C::LS + zl(c); };
  auto cload = [&](int e) { return buf[cidx(e)]; };
  for (int par = 0; par < 2; ++par) {
    if (par == 1) {
      // the even transforms' tile reads preceded their final barrier
#pragma unroll
      for (int j = 0; j < C::PER; ++j) buf[(r0 + C::OWN * j) * C::LS + zl(c)] = held(j);
      __syncthreads();
    }
    auto storeC = [&](int e, cx<T> v) {
      if (c == 0)
        pk[par * n + e] = v;
      else
        out[(x * N + 2 * e + par) * kp + c] = v;
    };
    fft_line<T, n, true>(r0, buf, cidx, tw, 2, cload, storeC);
  }
  __syncthreads();
  for (int i = t; i < 2 * n; i += C::THREADS) {
    const int par = i / n, e = i % n;
    const int em = par == 0 ? ((n - e) & (n - 1)) : (n - 1 - e);  // output -k
    const cx<T> cc = pk[i], cm = cconj<T>(pk[par * n + em]);
    const cx<T> s = cadd<T>(cc, cm), d = csub<T>(cc, cm);
    cx<T>* o = out + (x * N + 2 * e + par) * kp;
    o[0] = cscale<T>(s, half);
    o[n] = mkc<T>(half * d.y, -half * d.x);
  }
}

template <typename T, int N>
__global__ __launch_bounds__((ZYCfg<T, N>::THREADS)) void k_c2r_yz(
    const cx<T>* __restrict__ in, T* __restrict__ out, const cx<T>* __restrict__ twg, int kp) {
  using C = ZYCfg<T, N>;
  constexpr int n = C::n;
  __shared__ cx<T> buf[n * C::LS];
  __shared__ cx<T> tw[N];
  load_table<T>(tw, twg, N);  // visible after the first stage's barrier, before any use
  const int t = threadIdx.x;
  const size_t x = blockIdx.x;
  const int c = t % n, r0 = t / n;
  // held values: PER - 1 in registers, the last in LDS (the register file
  // is full)
  __shared__ cx<T> spare[C::THREADS];
  cx<T> keep[C::PER - 1];
  auto held = [&](int j) -> cx<T>& { return j < C::PER - 1 ? keep[j] : spare[t]; };
  auto cidx = [&](int e) { return e * C::LS + zl(c); };
  auto cstore = [&](int e, cx<T> v) { buf[cidx(e)] = v; };
  // inverse y transforms of the even and odd rows ky, the packed column
  // read as X(ky, 0) + i X(ky, n/2)
  for (int par = 0; par < 2; ++par) {
    auto load0 = [&](int e) -> cx<T> {  // both loads for every column: no branch
      const cx<T>* row = in + (x * N + 2 * e + par) * kp;
      const cx<T> u = row[c], v = row[n];
      return c != 0 ? u : mkc<T>(u.x - v.y, u.y + v.x);
    };
    fft_line<T, n, false>(r0, buf, cidx, tw, 2, load0, cstore);
    __syncthreads();
    if (par == 0) {
#pragma unroll
      for (int j = 0; j < C::PER; ++j) held(j) = buf[(r0 + C::OWN * j) * C::LS + zl(c)];
    }
    // the odd transforms' first tile store follows a barrier in fft_line
  }
  // radix-2 step: u(y) = E(y) + W^-y O(y), u(y + n) = E(y) - W^-y O(y)
#pragma unroll
  for (int j = 0; j < C::PER; ++j) {
    const int y = r0 + C::OWN * j;
    cx<T>* q = buf + y * C::LS + zl(c);
    const cx<T> o = cmul<T>(*q, cconj<T>(tw[y]));
    const cx<T> e = held(j);
    *q = cadd<T>(e, o);
    held(j) = csub<T>(e, o);
  }
  __syncthreads();
  const int lane = t % C::TPL, l = t / C::TPL;
  cx<T>* lb = buf + l * C::LS;
  // the real inverse's merge Z[e] = S + i W^-e D, S, D = X[e] +- conj X[n - e]
  auto merge = [&](cx<T> xk, cx<T> xc, int e) {
    const cx<T> s = cadd<T>(xk, xc);
    const cx<T> d = csub<T>(xk, xc);
    const cx<T> wd = cmul<T>(cconj<T>(tw[e]), d);
    return mkc<T>(s.x - wd.y, s.y + wd.x);
  };
  auto lidx = [&](int e) { return l * C::LS + zl(e); };
  auto lload = [&](int e) { return lb[zl(e)]; };
  for (int h = 0; h < 2; ++h) {
    if (h == 1) {
      // the first half's tile reads preceded the final barrier of its transform
#pragma unroll
      for (int j = 0; j < C::PER; ++j) buf[(r0 + C::OWN * j) * C::LS + zl(c)] = held(j);
      __syncthreads();
    }
    // merge in place, pair (k, n - k) by one thread; X[0] and X[n] (real)
    // packed in slot 0
    for (int k = lane; k <= n / 2; k += C::TPL) {
      const cx<T> xk = lb[zl(k)];
      if (k == 0) {
        lb[zl(0)] = merge(mkc<T>(xk.x, 0), mkc<T>(xk.y, 0), 0);
        continue;
      }
      const cx<T> xm = lb[zl(n - k)];
      lb[zl(k)] = merge(xk, cconj<T>(xm), k);
      if (k != n / 2) lb[zl(n - k)] = merge(xm, cconj<T>(xk), n - k);
    }
    __syncthreads();
    cx<T>* dst = reinterpret_cast<cx<T>*>(out + (x * N + h * n + l) * N);
    auto storeL = [&](int e, cx<T> v) { dst[e] = v; };
    fft_line<T, n, false>(lane, buf, lidx, tw, 2, lload, storeL);
  }
}

// ------------------------------------------------- strided C2C (y or x)
// Line L of the batch starts at (L / group) * gstride + L % group and its
// elements are estride apart; lines with L mod vmod >= vcnt are row padding
// and are skipped.
template <typename T, int N, bool FWD>
__global__ __launch_bounds__((SCfg<T, N>::THREADS)) void k_strided(
    const cx<T>* in, cx<T>* out, T scale, const cx<T>* __restrict__ twg, int nlines, int group,
    long long gstride, long long estride, int vmod, int vcnt) {
  using C = SCfg<T, N>;
  __shared__ cx<T> buf[N * C::LP];
  __shared__ cx<T> tw[N];
  load_table<T>(tw, twg, N);  // visible after the first stage's barrier, before any use
  const int l = threadIdx.x % C::LINES;
  const int lane = threadIdx.x / C::LINES;
  const int line = blockIdx.x * C::LINES + l;
  const bool valid = line < nlines && (line % vmod) < vcnt;
  const long long base = (long long)(line / group) * gstride + (line % group);
  auto load0 = [&](int e) -> cx<T> { return valid ? in[base + e * estride] : mkc<T>(0, 0); };
  auto storeL = [&](int e, cx<T> v) {
    if (valid) out[base + e * estride] = cscale<T>(v, scale);
  };
  auto lidx = [&](int e) { return e * C::LP + l; };
  fft_line<T, N, FWD>(lane, buf, lidx, tw, 1, load0, storeL);
}

// ------------------------------------------------- k-space multipliers
// Integer wavenumber of index i on a full axis of side N and its derivative
// version (0 at the Nyquist index).
__device__ __forceinline__ int wave_index(int i, int N) { return i < N / 2 ? i : i - N; }

// Component a (0, 1, 2) of an integer wave vector; a is the same for the
// whole workgroup, so this is a select, not an indexed (private memory) load.
__device__ __forceinline__ int pick(int a, int kx, int ky, int kz) {
  return a == 0 ? kx : (a == 1 ? ky : kz);
}

// Multiplier j of ms applied to v at wave vector (kx, ky, kz) in units of the
// fundamental mode (derivative versions), n2 = |k|^2 in the same units.
template <typename T>
__device__ __forceinline__ cx<T> apply_mult(cx<T> v, const MulSet& ms, int j, int n2, int kx,
                                            int ky, int kz, const T* __restrict__ wtab,
                                            T L_over_2pi) {
  const int kinds = ms.kinds[j];
  T f = static_cast<T>(ms.scale[j]);
  if (kinds == 0) return cscale<T>(v, f);
  if (n2 == 0) return mkc<T>(0, 0);
  if (kinds & MUL_WHITE) f *= wtab[n2];
  const T inv = static_cast<T>(1) / static_cast<T>(n2);
  if (kinds & MUL_HESS)
    f *= static_cast<T>(pick(ms.ha[j], kx, ky, kz) * pick(ms.hb[j], kx, ky, kz)) * inv;
  if (kinds & MUL_GRAD) {
    f *= L_over_2pi * static_cast<T>(pick(ms.ga[j], kx, ky, kz)) * inv;
    return mkc<T>(-v.y * f, v.x * f);  // i f v
  }
  return cscale<T>(v, f);
}

template <typename T>
struct OutPtrs {
  cx<T>* p[kMaxMul];
};
template <typename T>
struct InPtrs {
  const cx<T>* p[kMaxMul];
};

// Forward x FFT, then m inverse x FFTs of the multiplied spectrum; the
// forward result stays in registers (XPlan layout) across the m inverses.
template <typename T, int N>
__global__ __launch_bounds__((FCfg<T, N>::THREADS), (FCfg<T, N>::MINW)) void k_x_scatter(
    const cx<T>* __restrict__ in, OutPtrs<T> outs, MulSet ms, int m,
    const T* __restrict__ wtab, T L_over_2pi, const cx<T>* __restrict__ twg, int nlines,
    int K, int kp) {
  using C = FCfg<T, N>;
  using X = XPlan<N>;
  __shared__ cx<T> B[N * C::LP];
  __shared__ cx<T> tw[N];
  load_table<T>(tw, twg, N);  // visible after the first stage's barrier, before any use
  const int l = threadIdx.x % C::LINES;
  const int lane = threadIdx.x / C::LINES;
  const int line = blockIdx.x * C::LINES + l;
  const int ky = line / kp, kz = line % kp;
  const bool valid = line < nlines && kz < K;
  const long long stride = (long long)nlines;  // = N * kp
  const int iy = wave_index(ky, N), iz = kz;
  const int dy = (ky == N / 2) ? 0 : iy, dz = (kz == N / 2) ? 0 : iz;
  auto lidx = [&](int e) { return e * C::LP + l; };
  auto load_in = [&](int e) -> cx<T> { return valid ? in[line + e * stride] : mkc<T>(0, 0); };
  cx<T> V[X::BPT][X::RL];
  fft_fwd_to_regs<T, N, PlanX<N>>(lane, B, lidx, tw, load_in, V);
  for (int j = 0; j < m; ++j) {
    cx<T> W[X::BPT][X::RL];
#pragma unroll
    for (int b = 0; b < X::BPT; ++b) {
#pragma unroll
      for (int r = 0; r < X::RL; ++r) {
        const int e = lane + b * X::TPL + r * X::NBL;
        const int ix = wave_index(e, N);
        const int n2 = ix * ix + iy * iy + iz * iz;
        W[b][r] = apply_mult<T>(V[b][r], ms, j, n2, (e == N / 2) ? 0 : ix, dy, dz, wtab,
                                L_over_2pi);
      }
    }
    cx<T>* dst = outs.p[j];
    auto store_o = [&](int e, cx<T> v) {
      if (valid) dst[line + e * stride] = v;
    };
    fft_inv_from_regs<T, N, PlanX<N>>(lane, B, lidx, tw, W, store_o);
  }
}

// Sum over m inputs of multiplier * forward x FFT (accumulated in
// registers), then one inverse x FFT.
template <typename T, int N>
__global__ __launch_bounds__((FCfg<T, N, PlanG<N>>::THREADS)) void k_x_gather(
    InPtrs<T> ins, MulSet ms, int m, cx<T>* out, const T* __restrict__ wtab, T L_over_2pi,
    const cx<T>* __restrict__ twg, int nlines, int K, int kp) {
  using C = FCfg<T, N, PlanG<N>>;
  using X = XPlan<N, PlanG<N>>;
  __shared__ cx<T> B[N * C::LP];
  __shared__ cx<T> tw[N];
  load_table<T>(tw, twg, N);  // visible after the first stage's barrier, before any use
  const int l = threadIdx.x % C::LINES;
  const int lane = threadIdx.x / C::LINES;
  const int line = blockIdx.x * C::LINES + l;
  const int ky = line / kp, kz = line % kp;
  const bool valid = line < nlines && kz < K;
  const long long stride = (long long)nlines;  // = N * kp
  const int iy = wave_index(ky, N), iz = kz;
  const int dy = (ky == N / 2) ? 0 : iy, dz = (kz == N / 2) ? 0 : iz;
  auto lidx = [&](int e) { return e * C::LP + l; };
  cx<T> acc[X::BPT][X::RL];
  for (int j = 0; j < m; ++j) {
    const cx<T>* src = ins.p[j];
    auto load_in = [&](int e) -> cx<T> {
      return valid ? src[line + e * stride] : mkc<T>(0, 0);
    };
    cx<T> V[X::BPT][X::RL];
    fft_fwd_to_regs<T, N, PlanG<N>>(lane, B, lidx, tw, load_in, V);
#pragma unroll
    for (int b = 0; b < X::BPT; ++b) {
#pragma unroll
      for (int r = 0; r < X::RL; ++r) {
        const int e = lane + b * X::TPL + r * X::NBL;
        const int ix = wave_index(e, N);
        const int n2 = ix * ix + iy * iy + iz * iz;
        const cx<T> t = apply_mult<T>(V[b][r], ms, j, n2, (e == N / 2) ? 0 : ix, dy, dz, wtab,
                                      L_over_2pi);
        acc[b][r] = j == 0 ? t : cadd<T>(acc[b][r], t);
      }
    }
  }
  auto store_o = [&](int e, cx<T> v) {
    if (valid) out[line + e * stride] = v;
  };
  fft_inv_from_regs<T, N, PlanG<N>>(lane, B, lidx, tw, acc, store_o);
}

// ------------------------------------------------- layout conversion
// Copies between the stored half spectrum (row pitch kp) and the contiguous
// [n][n][n/2+1] layout; pack = stored -> contiguous.
template <typename T, bool PACK>
__global__ void k_spec_copy(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int K,
                            int kp, long long H) {
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < H;
       f += (long long)gridDim.x * blockDim.x) {
    const long long s = (f / K) * kp + f % K;
    if (PACK)
      dst[f] = src[s];
    else
      dst[s] = src[f];
  }
}

// ------------------------------------------------------------ dispatch
// f(ZH, B) with the two flags as compile-time constants.
template <class F>
void with_flags(bool zh, bool b, F&& f) {
  using Y = std::true_type;
  using No = std::false_type;
  if (zh) {
    if (b)
      f(Y{}, Y{});
    else
      f(Y{}, No{});
  } else {
    if (b)
      f(No{}, Y{});
    else
      f(No{}, No{});
  }
}

template <typename T, class F>
void dispatch_n(int n, F&& f) {
  switch (n) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    default: throw ApiError(-2, "FFT size must be a power of two in [8, 1024]");
  }
}

inline MulSet make_set(const MulSpec* specs, int m) {
  if (m < 1 || m > kMaxMul) throw ApiError(-1, "multiplier count out of range");
  MulSet s{};
  for (int j = 0; j < m; ++j) {
    s.kinds[j] = specs[j].kinds;
    s.ga[j] = specs[j].ga;
    s.ha[j] = specs[j].ha;
    s.hb[j] = specs[j].hb;
    s.scale[j] = specs[j].scale;
  }
  return s;
}

}  // namespace fftk

template <typename T>
void fft_r2c_z(const FftArgs<T>& f, const T* a, T alpha, const T* b, T beta, cx<T>* out,
               const T* zh) {
  fftk::dispatch_n<T>(f.n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = fftk::ZCfg<T, N>;
    const int nlines = f.n * f.n;
    fftk::with_flags(zh != nullptr, b != nullptr, [&](auto ZH, auto B) {
      fftk::k_r2c_z<T, N, ZH.value, B.value>
          <<<blocks_for(nlines, C::LINES), C::THREADS, 0, f.stream>>>(a, alpha, b, beta, out,
                                                                      f.tw, nlines, f.kp, zh);
    });
  });
  IC_LAUNCHED();
}

template <typename T>
void fft_c2r_z(const FftArgs<T>& f, const cx<T>* in, T* out, T alpha, const T* aux, T beta) {
  fftk::dispatch_n<T>(f.n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = fftk::ZCfg<T, N>;
    const int nlines = f.n * f.n;
    fftk::k_c2r_z<T, N><<<blocks_for(nlines, C::LINES), C::THREADS, 0, f.stream>>>(
        in, out, alpha, aux, beta, f.tw, nlines, f.kp);
  });
  IC_LAUNCHED();
}

template <typename T>
bool fft_zy_fused(int n) {
  return fftk::ZYCfg<T, 256>::ok && n == 256;
}

template <typename T>
void fft_r2c_zy(const FftArgs<T>& f, const T* a, T alpha, const T* b, T beta, cx<T>* out,
                const T* zh) {
  if constexpr (fftk::ZYCfg<T, 256>::ok) {
    if (f.n == 256) {
      using C = fftk::ZYCfg<T, 256>;
      fftk::with_flags(zh != nullptr, b != nullptr, [&](auto ZH, auto B) {
        fftk::k_r2c_zy<T, 256, ZH.value, B.value>
            <<<f.n, C::THREADS, 0, f.stream>>>(a, alpha, b, beta, out, f.tw, f.kp, zh);
      });
      IC_LAUNCHED();
      return;
    }
  }
  throw ApiError(-2, "fused z and y passes: FP32 at n = 256 only");
}

template <typename T>
void fft_c2r_yz(const FftArgs<T>& f, const cx<T>* in, T* out) {
  if constexpr (fftk::ZYCfg<T, 256>::ok) {
    if (f.n == 256) {
      using C = fftk::ZYCfg<T, 256>;
      fftk::k_c2r_yz<T, 256><<<f.n, C::THREADS, 0, f.stream>>>(in, out, f.tw, f.kp);
      IC_LAUNCHED();
      return;
    }
  }
  throw ApiError(-2, "fused y and z passes: FP32 at n = 256 only");
}

template <typename T>
void fft_y(const FftArgs<T>& f, cx<T>* data, bool forward) {
  fftk::dispatch_n<T>(f.n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = fftk::SCfg<T, N>;
    const int K = N / 2 + 1, kp = f.kp;
    const int nlines = N * kp;
    const unsigned grid = blocks_for(nlines, C::LINES);
    if (forward)
      fftk::k_strided<T, N, true><<<grid, C::THREADS, 0, f.stream>>>(
          data, data, T(1), f.tw, nlines, kp, (long long)N * kp, kp, kp, K);
    else
      fftk::k_strided<T, N, false><<<grid, C::THREADS, 0, f.stream>>>(
          data, data, T(1), f.tw, nlines, kp, (long long)N * kp, kp, kp, K);
  });
  IC_LAUNCHED();
}

template <typename T>
void fft_x(const FftArgs<T>& f, const cx<T>* in, cx<T>* out, bool forward, T scale) {
  fftk::dispatch_n<T>(f.n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = fftk::SCfg<T, N>;
    const int K = N / 2 + 1, kp = f.kp;
    const int nlines = N * kp;
    const unsigned grid = blocks_for(nlines, C::LINES);
    if (forward)
      fftk::k_strided<T, N, true><<<grid, C::THREADS, 0, f.stream>>>(
          in, out, scale, f.tw, nlines, nlines, 0, nlines, kp, K);
    else
      fftk::k_strided<T, N, false><<<grid, C::THREADS, 0, f.stream>>>(
          in, out, scale, f.tw, nlines, nlines, 0, nlines, kp, K);
  });
  IC_LAUNCHED();
}

template <typename T>
void spectrum_pack(const FftArgs<T>& f, const cx<T>* stored, cx<T>* dense) {
  const int K = f.n / 2 + 1;
  const long long H = (long long)f.n * f.n * K;
  fftk::k_spec_copy<T, true><<<grid_for(H, 256), 256, 0, f.stream>>>(stored, dense, K, f.kp, H);
  IC_LAUNCHED();
}

template <typename T>
void spectrum_unpack(const FftArgs<T>& f, const cx<T>* dense, cx<T>* stored) {
  const int K = f.n / 2 + 1;
  const long long H = (long long)f.n * f.n * K;
  fftk::k_spec_copy<T, false><<<grid_for(H, 256), 256, 0, f.stream>>>(dense, stored, K, f.kp, H);
  IC_LAUNCHED();
}

template <typename T>
void fft_x_scatter(const FftArgs<T>& f, const cx<T>* in, cx<T>* const* outs,
                   const MulSpec* specs, int m) {
  MulSet ms = fftk::make_set(specs, m);
  fftk::OutPtrs<T> op{};
  for (int j = 0; j < m; ++j) op.p[j] = outs[j];
  const T l2p = static_cast<T>(f.box / (2.0 * 3.14159265358979323846));
  fftk::dispatch_n<T>(f.n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = fftk::FCfg<T, N>;
    const int K = N / 2 + 1;
    const int nlines = N * f.kp;
    fftk::k_x_scatter<T, N><<<blocks_for(nlines, C::LINES), C::THREADS, 0, f.stream>>>(
        in, op, ms, m, f.wtab, l2p, f.tw, nlines, K, f.kp);
  });
  IC_LAUNCHED();
}

template <typename T>
void fft_x_gather(const FftArgs<T>& f, const cx<T>* const* ins, const MulSpec* specs, int m,
                  cx<T>* out) {
  MulSet ms = fftk::make_set(specs, m);
  fftk::InPtrs<T> ip{};
  for (int j = 0; j < m; ++j) ip.p[j] = ins[j];
  const T l2p = static_cast<T>(f.box / (2.0 * 3.14159265358979323846));
  fftk::dispatch_n<T>(f.n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = fftk::FCfg<T, N, fftk::PlanG<N>>;
    const int K = N / 2 + 1;
    const int nlines = N * f.kp;
    fftk::k_x_gather<T, N><<<blocks_for(nlines, C::LINES), C::THREADS, 0, f.stream>>>(
        ip, ms, m, out, f.wtab, l2p, f.tw, nlines, K, f.kp);
  });
  IC_LAUNCHED();
}

}  // namespace ic
