// The stable descending sort of rank-order matching (section 2.3.2, step 1:
// the rank of every element) for callers that cannot allocate device
// memory: the radix sort's keys, indices and digit histograms live in one
// file-scope device array instead of a context workspace.  The kernels are
// the context path's own (sort.h).
#include <mutex>

#include "../../include/ic_ops.h"
#include "sort.h"

namespace ic {
namespace na {

constexpr long long kMaxN = IC_NOALLOC_SORT_MAX;
constexpr long long kTiles = (kMaxN + sk::kTile - 1) / sk::kTile;
// keys, keys (ping-pong), indices, indices (ping-pong), histogram, NaN count
constexpr size_t kKeysOff = 0;
constexpr size_t kKeys2Off = kKeysOff + 8 * kMaxN;
constexpr size_t kValsOff = kKeys2Off + 8 * kMaxN;
constexpr size_t kVals2Off = kValsOff + 4 * kMaxN;
constexpr size_t kHistOff = kVals2Off + 4 * kMaxN;
constexpr size_t kCountOff = (kHistOff + 4 * sk::kDigits * kTiles + 255) & ~size_t(255);
constexpr size_t kScratchBytes = kCountOff + 256;

// Each device that runs the entry point holds its own copy until the
// process ends.  In host code the name is a host-side stand-in: only the
// address returned by hipGetSymbolAddress may reach a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current).
void* scratch_address() {
  int dev = -1;
  IC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw ApiError(IC_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    IC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ApiError(IC_ERR_HIP, "no device address for the sort scratch");
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// Count of NaN values added into *count (zeroed by k_zero_u32 first: the
// array keeps the previous call's contents).
template <typename T>
__global__ __launch_bounds__(256) void k_count_nan(const T* __restrict__ x, long long n,
                                                   unsigned* __restrict__ count) {
  unsigned c = 0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    c += x[i] != x[i];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void k_zero_u32(unsigned* __restrict__ x) { *x = 0u; }

template <typename T>
void sort_desc(const T* values, long long n, int32_t* order, hipStream_t st) {
  char* base = static_cast<char*>(scratch_address());
  uint64_t* keys = reinterpret_cast<uint64_t*>(base + kKeysOff);
  uint64_t* keys2 = reinterpret_cast<uint64_t*>(base + kKeys2Off);
  uint32_t* vals = reinterpret_cast<uint32_t*>(base + kValsOff);
  uint32_t* vals2 = reinterpret_cast<uint32_t*>(base + kVals2Off);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + kHistOff);
  unsigned* count = reinterpret_cast<unsigned*>(base + kCountOff);
  k_zero_u32<<<1, 1, 0, st>>>(count);
  IC_LAUNCHED();
  k_count_nan<T><<<grid_for(n, 256, 1024), 256, 0, st>>>(values, n, count);
  IC_LAUNCHED();
  unsigned nan = 0;
  IC_HIP(hipMemcpyAsync(&nan, count, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  IC_HIP(hipStreamSynchronize(st));
  if (nan) throw ApiError(IC_ERR_NONFINITE, "NaN in sort input");
  sk::k_desc_keys<T><<<grid_for(n, 256), 256, 0, st>>>(values, keys, vals, n);
  IC_LAUNCHED();
  radix_sort_pairs(keys, vals, keys2, vals2, hist, n, 8 * sizeof(T), st);
  IC_HIP(hipMemcpyAsync(order, vals, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
}

}  // namespace na
}  // namespace ic

namespace ic {

void noalloc_sort_desc(int precision, const void* values, int64_t n, int32_t* order,
                       hipStream_t st) {
  if (n < 0 || n > IC_NOALLOC_SORT_MAX)
    throw ApiError(IC_ERR_INVALID_ARG, "sort length must be in [0, IC_NOALLOC_SORT_MAX = 2^21]");
  if (precision != IC_F32 && precision != IC_F64)
    throw ApiError(IC_ERR_INVALID_ARG, "precision must be IC_F32 or IC_F64");
  if (n == 0) return;
  if (!values || !order) throw ApiError(IC_ERR_INVALID_ARG, "null buffer");
  if (precision == IC_F32)
    na::sort_desc<float>(static_cast<const float*>(values), n, order, st);
  else
    na::sort_desc<double>(static_cast<const double*>(values), n, order, st);
}

}  // namespace ic
