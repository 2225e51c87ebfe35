// Shared device/host helpers of the MI355X (gfx950) hot-path library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace ic {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
// Interleaved complex number of precision T (re in .x, im in .y).
template <typename T> using cx = typename Vec2<T>::type;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mkc(T re, T im) {
  cx<T> r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return mkc<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return mkc<T>(a.x - b.x, a.y - b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mkc<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cconj(cx<T> a) {
  return mkc<T>(a.x, -a.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return mkc<T>(a.x * s, a.y * s);
}

// Thrown by host code on a failed HIP call; the C ABI turns it into IC_ERR_HIP.
struct HipError : std::runtime_error {
  explicit HipError(const std::string& m) : std::runtime_error(m) {}
};
// Thrown for invalid arguments / unsupported shapes / state errors.
struct ApiError : std::runtime_error {
  int code;
  ApiError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    throw HipError(std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file +
                   ":" + std::to_string(line) + ")");
  }
}
#define IC_HIP(call) ::ic::hip_check((call), #call, __FILE__, __LINE__)
#define IC_LAUNCHED() ::ic::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

inline unsigned blocks_for(size_t n, unsigned threads) {
  return static_cast<unsigned>((n + threads - 1) / threads);
}

// Grid-stride element count helper: enough blocks to fill the chip without
// exceeding the element count.
inline unsigned grid_for(size_t n, unsigned threads, unsigned cap = 8192) {
  size_t b = (n + threads - 1) / threads;
  if (b > cap) b = cap;
  if (b == 0) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace ic
