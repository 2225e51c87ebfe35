// Lagrangian particle tiles with LDS-staged mesh windows (gfx950).
//
// One 256-thread workgroup owns a 4 x 8 x 16 block of lattice particles
// (two per thread).  Because particles move a few cells at most relative to
// their lattice neighbours, the CIC stencils of a tile fall inside a small
// Eulerian box.  The workgroup finds that box (LDS min/max), and then
//   * paints into an LDS window with LDS atomics and flushes each non-zero
//     window cell to HBM with one global atomic, consecutive lanes on
//     consecutive cells so a wavefront's atomics fall on few cache lines;
//   * or reads mesh fields for gathers from a window loaded with coalesced
//     row loads, so every CIC corner read is an LDS read.
// Paint windows accumulate in FP64 for both precisions: on gfx950 the LDS
// FP64 atomic add (ds_add_f64) sustains about twenty times the lane rate of
// the FP32 one (ds_add_f32), which executes close to one lane at a time, and
// the FP64 sum is rounded to the mesh precision once, at the flush.
// A tile whose box exceeds the window capacity (strongly clustered regions)
// takes the direct global path for that call; results agree to rounding.
#pragma once

#include <climits>

#include "particles.h"

namespace ic {
namespace tk {

constexpr int kThreads = 256;
constexpr int kPer = 2;  // particles per thread
constexpr int kWCap = 4096;  // window cells per field

// FP64 paint-window accumulator.
using Acc = double;

// Bytes of a kernel's LDS block holding ng gather fields of T, or one paint
// window of Acc, whichever is larger (the two phases reuse the block).
template <typename T>
constexpr unsigned lds_bytes(int ng) {
  const unsigned g = (unsigned)(ng * kWCap) * (unsigned)sizeof(T);
  const unsigned p = (unsigned)kWCap * (unsigned)sizeof(Acc);
  return g > p ? g : p;
}

// Tile shape (tx, ty, tz) and tile counts per axis for a side-n lattice.
struct TileGeom {
  int tx, ty, tz;
  int nx, ny, nz;
};

inline TileGeom tile_geom(int n) {
  TileGeom t;
  t.tx = n < 4 ? n : 4;
  t.ty = n < 8 ? n : 8;
  t.tz = n < 16 ? n : 16;
  t.nx = n / t.tx;
  t.ny = n / t.ty;
  t.nz = n / t.tz;
  return t;
}

inline unsigned tile_count(const TileGeom& t) { return (unsigned)(t.nx * t.ny * t.nz); }

// Workgroups are dealt to the eight XCDs round-robin (block b runs on XCD
// b mod 8).  Tile t = (b mod 8) * (count / 8) + b / 8 gives each XCD one
// contiguous slab of tiles, so the halo cache lines that neighbouring tiles
// share are read and updated in the same L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int b, int count) {
  if (count % kXcds != 0) return b;
  return (b % kXcds) * (count / kXcds) + b / kXcds;
}

// Particle slot k of this thread: lattice index and flat index; false when
// the slot is outside the tile.
__device__ __forceinline__ bool tile_particle(const TileGeom& tg, int lp, int k, int idx[3],
                                              long long& n) {
  const int l = threadIdx.x + k * kThreads;
  const int cnt = tg.tx * tg.ty * tg.tz;
  if (l >= cnt) return false;
  const int lz = l % tg.tz, ly = (l / tg.tz) % tg.ty, lx = l / (tg.tz * tg.ty);
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int bz = b % tg.nz, by = (b / tg.nz) % tg.ny, bx = b / (tg.nz * tg.ny);
  idx[0] = bx * tg.tx + lx;
  idx[1] = by * tg.ty + ly;
  idx[2] = bz * tg.tz + lz;
  n = ((long long)idx[0] << (2 * lp)) | ((long long)idx[1] << lp) | (long long)idx[2];
  return true;
}

// Eulerian window (unwrapped cell coordinates) covering a set of stencils.
struct Window {
  int o[3];
  int w[3];
  int vol;
  bool fits;
};

struct BoxShared {
  int lo[3];
  int hi[3];
};

__device__ __forceinline__ void box_init(BoxShared& b) {
  if (threadIdx.x < 3) {
    b.lo[threadIdx.x] = INT_MAX;
    b.hi[threadIdx.x] = INT_MIN;
  }
}

// Adds this thread's range lo .. hi (per axis) to the box: reduced across
// the wavefront with shuffles first, so each wave issues one LDS atomic per
// bound instead of 64 contending ones.
__device__ __forceinline__ void box_add_range(BoxShared& b, int lo[3], int hi[3]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], __shfl_xor(lo[a], off, 64));
      hi[a] = max(hi[a], __shfl_xor(hi[a], off, 64));
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(&b.lo[a], lo[a]);
      atomicMax(&b.hi[a], hi[a]);
    }
  }
}

// Call after a barrier that follows all box_add calls.
__device__ __forceinline__ Window box_window(const BoxShared& b) {
  Window w;
  long long vol = 1;
  bool empty = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w.o[a] = b.lo[a];
    const long long ext = (long long)b.hi[a] - (long long)b.lo[a] + 1;
    if (ext <= 0) empty = true;
    w.w[a] = ext > 0 && ext < (1 << 20) ? static_cast<int>(ext) : 0;
    vol *= ext > 0 ? ext : 0;
  }
  w.fits = !empty && vol <= kWCap;
  w.vol = w.fits ? static_cast<int>(vol) : 0;
  return w;
}

// Window-local index of unwrapped cell c.
__device__ __forceinline__ int win_index(const Window& w, int cx, int cy, int cz) {
  return ((cx - w.o[0]) * w.w[1] + (cy - w.o[1])) * w.w[2] + (cz - w.o[2]);
}

// Physical (wrapped) mesh index of window cell number k.
__device__ __forceinline__ long long win_cell(const Window& w, int k, int mask, int lm) {
  const int cz = w.o[2] + k % w.w[2];
  const int t = k / w.w[2];
  const int cy = w.o[1] + t % w.w[1];
  const int cx = w.o[0] + t / w.w[1];
  const int c[3] = {cx, cy, cz};
  return pk::cell_index(c, mask, lm);
}

// Loads nf fields (stride M) of the window into lds[f * kWCap + k].  Each
// thread issues the loads of kBatch cells before storing any of them, so the
// loads of a batch are in flight together instead of one at a time.
constexpr int kBatch = 8;

template <typename T>
__device__ __forceinline__ void win_load(const Window& w, const T* __restrict__ src, long long M,
                                         int nf, int lm, T* lds) {
  const int mask = (1 << lm) - 1;
  for (int base = 0; base < w.vol; base += kBatch * kThreads) {
    T v[kBatch][4];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = base + j * kThreads + threadIdx.x;
      if (k < w.vol) {
        const long long c = win_cell(w, k, mask, lm);
#pragma unroll
        for (int f = 0; f < 4; ++f)
          if (f < nf) v[j][f] = src[f * M + c];
      }
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = base + j * kThreads + threadIdx.x;
      if (k < w.vol) {
#pragma unroll
        for (int f = 0; f < 4; ++f)
          if (f < nf) lds[f * kWCap + k] = v[j][f];
      }
    }
  }
}

__device__ __forceinline__ void win_zero(const Window& w, Acc* acc) {
  for (int k = threadIdx.x; k < w.vol; k += kThreads) acc[k] = Acc(0);
}

// Adds the non-zero cells of one FP64 window into the mesh of type T with
// global atomics.  Consecutive lanes take consecutive window cells (rows run
// along z), so a wavefront's atomics fall on a few cache lines: the memory
// system applies all lanes that hit one line in a single operation, which is
// what makes the flush cheap compared with one atomic stream per particle.
template <typename T>
__device__ __forceinline__ void win_flush(const Window& w, const Acc* acc, int lm,
                                          T* __restrict__ dst) {
  const int mask = (1 << lm) - 1;
  for (int base = 0; base < w.vol; base += kBatch * kThreads) {
    T v[kBatch];
    long long c[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = base + j * kThreads + threadIdx.x;
      c[j] = -1;
      if (k < w.vol) {
        c[j] = win_cell(w, k, mask, lm);
        v[j] = static_cast<T>(acc[k]);
      }
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (c[j] >= 0 && v[j] != T(0)) pk::atomic_add(dst + c[j], v[j]);
  }
}

// Counts tiles that did not fit their window (they took the direct path).
__device__ __forceinline__ void count_overflow(const Window& w, unsigned* counter) {
  if (!w.fits && counter && threadIdx.x == 0) atomicAdd(counter, 1u);
}

}  // namespace tk
}  // namespace ic
