// Host interface of the LDS-staged Stockham FFT passes (gfx950).
//
// A 3D real transform of an n^3 cube is three axis passes: a real-to-complex
// pass along the contiguous z axis (half-length complex FFT plus the
// even/odd split), and complex passes along y and x over the half spectrum
// [n][n][n/2+1], stored with each z row padded to kp >= n/2+1 entries so
// that rows start on 128-byte boundaries and the strided passes move whole
// cache lines (the pad entries are never read).  The x pass is the last forward axis
// and the first inverse one, so k-space multipliers are applied inside it:
// one kernel runs the forward x FFT, multiplies by m multipliers and runs m
// inverse x FFTs (scatter), or the reverse for m inputs summed into one
// output (gather).  Inverse passes are unnormalised; the 1/n^3 of the
// inverse real DFT is folded into the multiplier scale.  For FP32 at n = 256
// the z and y passes also run fused, one x plane per workgroup.
#pragma once

#include "common.h"

namespace ic {

enum MulKind : int { MUL_WHITE = 1, MUL_GRAD = 2, MUL_HESS = 4 };

// One k-space multiplier: scale * [w(k)] * [i k~_ga / k^2] * [k~_ha k~_hb / k^2].
// With no kind bits it is the plain scale (the k = 0 mode kept); otherwise it
// vanishes at k = 0.
struct MulSpec {
  int kinds = 0;
  int ga = 0, ha = 0, hb = 0;
  double scale = 1.0;
};

constexpr int kMaxMul = 9;
// Spacing along z of the cells that receive a paint's z halo (the block side
// of the particle orders).
constexpr int kZHalo = 8;

struct MulSet {
  int kinds[kMaxMul];
  int ga[kMaxMul];
  int ha[kMaxMul];
  int hb[kMaxMul];
  double scale[kMaxMul];
};

// Row pitch of the stored half spectrum: n/2+1 rounded up to a multiple of
// 128 bytes.
template <typename T>
inline int spectrum_pitch(int n) {
  const int q = 128 / static_cast<int>(sizeof(cx<T>));
  const int k = n / 2 + 1;
  return (k + q - 1) / q * q;
}

template <typename T>
struct FftArgs {
  int n = 0;                    // grid side
  int kp = 0;                   // stored row pitch of the half spectrum (spectrum_pitch)
  const cx<T>* tw = nullptr;    // device table exp(-2 pi i m / n), m < n
  const T* wtab = nullptr;      // whitening multiplier indexed by |k|^2 / kf^2 (particle grid)
  double box = 1.0;             // box side (for i k / k^2)
  hipStream_t stream = nullptr;
};

// out = forward rfft along z of (alpha a + beta b); b may be null.
template <typename T>
void fft_r2c_z(const FftArgs<T>& f, const T* a, T alpha, const T* b, T beta, cx<T>* out,
               const T* zh = nullptr);

// out = alpha * (unnormalised inverse rfft along z of in) + beta * aux (aux may be null).
template <typename T>
void fft_c2r_z(const FftArgs<T>& f, const cx<T>* in, T* out, T alpha, const T* aux, T beta);

// Whether the fused z and y passes below serve grid side n at this precision.
template <typename T>
bool fft_zy_fused(int n);

// fft_r2c_z then the forward fft_y in one pass (where fft_zy_fused).
template <typename T>
void fft_r2c_zy(const FftArgs<T>& f, const T* a, T alpha, const T* b, T beta, cx<T>* out,
                const T* zh = nullptr);

// The inverse fft_y then fft_c2r_z (alpha 1, no aux) in one pass (where
// fft_zy_fused), for the spectrum of a real field: its kz = 0 and kz = n/2
// columns must be Hermitian along y (their inverse along y real).
template <typename T>
void fft_c2r_yz(const FftArgs<T>& f, const cx<T>* in, T* out);

// In-place complex FFT along y of the half spectrum (forward or inverse, unnormalised).
template <typename T>
void fft_y(const FftArgs<T>& f, cx<T>* data, bool forward);

// Complex FFT along x, out = scale * FFT(in); in may equal out.
template <typename T>
void fft_x(const FftArgs<T>& f, const cx<T>* in, cx<T>* out, bool forward, T scale);

// Copies between the stored half spectrum and the contiguous n x n x (n/2+1) layout.
template <typename T>
void spectrum_pack(const FftArgs<T>& f, const cx<T>* stored, cx<T>* dense);
template <typename T>
void spectrum_unpack(const FftArgs<T>& f, const cx<T>* dense, cx<T>* stored);

// Forward x FFT of in, then for each j < m: outs[j] = inverse x FFT of (mult_j * .).
template <typename T>
void fft_x_scatter(const FftArgs<T>& f, const cx<T>* in, cx<T>* const* outs,
                   const MulSpec* specs, int m);

// out = inverse x FFT of sum_j mult_j * forward x FFT of ins[j]; out may equal ins[0].
template <typename T>
void fft_x_gather(const FftArgs<T>& f, const cx<T>* const* ins, const MulSpec* specs, int m,
                  cx<T>* out);

}  // namespace ic
