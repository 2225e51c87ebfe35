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
#ifndef IC_TILE_GCAP
#define IC_TILE_GCAP 2048
#endif
#ifndef IC_TILE_PCAP
#define IC_TILE_PCAP 4096
#endif
#ifndef IC_TILE_WAVES
#define IC_TILE_WAVES 1
#endif
// Window capacities in cells: per field for gather windows (mesh type), and
// for the one FP64 paint window.  A direct-path gather costs little more than
// a window gather while a direct-path paint costs one global atomic per
// corner, so paint windows get the larger capacity.
constexpr int kGCap = IC_TILE_GCAP;
constexpr int kPCap = IC_TILE_PCAP;
constexpr int kWaves = IC_TILE_WAVES;  // minimum waves per SIMD asked of the compiler

// FP64 paint-window accumulator.
using Acc = double;

// Bytes of a kernel's LDS block holding ng gather fields of T, or one paint
// window of Acc, whichever is larger (the two phases reuse the block).
template <typename T>
constexpr unsigned lds_bytes(int ng) {
  const unsigned g = (unsigned)(ng * kGCap) * (unsigned)sizeof(T);
  const unsigned p = (unsigned)kPCap * (unsigned)sizeof(Acc);
  return g > p ? g : p;
}

// Tile shape (tx, ty, tz) and tile counts per axis for a side-n lattice,
// with their base-2 logarithms (every extent is a power of two).
struct TileGeom {
  int tx, ty, tz;
  int nx, ny, nz;
  int ltx, lty, ltz;
  int lnx, lny, lnz;
};

inline int tile_log2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline TileGeom tile_geom(int n) {
  TileGeom t;
  t.tx = n < 4 ? n : 4;
  t.ty = n < 8 ? n : 8;
  t.tz = n < 16 ? n : 16;
  t.nx = n / t.tx;
  t.ny = n / t.ty;
  t.nz = n / t.tz;
  t.ltx = tile_log2(t.tx);
  t.lty = tile_log2(t.ty);
  t.ltz = tile_log2(t.tz);
  t.lnx = tile_log2(t.nx);
  t.lny = tile_log2(t.ny);
  t.lnz = tile_log2(t.nz);
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
  if (l >> (tg.ltx + tg.lty + tg.ltz)) return false;
  const int lz = l & (tg.tz - 1), ly = (l >> tg.ltz) & (tg.ty - 1), lx = l >> (tg.ltz + tg.lty);
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int bz = b & (tg.nz - 1), by = (b >> tg.lnz) & (tg.ny - 1), bx = b >> (tg.lnz + tg.lny);
  idx[0] = (bx << tg.ltx) + lx;
  idx[1] = (by << tg.lty) + ly;
  idx[2] = (bz << tg.ltz) + lz;
  n = ((long long)idx[0] << (2 * lp)) | ((long long)idx[1] << lp) | (long long)idx[2];
  return true;
}

// Eulerian window (unwrapped cell coordinates) covering a set of stencils.
struct Window {
  int o[3];
  int w[3];
  int vol;
  bool fits;
  unsigned mz, my;  // division magics of w[2] and w[1] (div_magic)
};

// floor(k / d) for d >= 2 as the high word of k * ceil(2^32 / d): exact
// whenever k * d < 2^32, which holds for window indices and extents (both
// below 2^16).  ceil(2^32 / d) is computed in FP64, exact because 2^32 / d
// is either an integer or at least 1/d away from one.  d = 1 maps to 0 and
// is handled by div_by.
__device__ __forceinline__ unsigned div_magic(int d) {
  return d > 1 ? static_cast<unsigned>(ceil(4294967296.0 / static_cast<double>(d))) : 0u;
}
__device__ __forceinline__ int div_by(int k, unsigned m) {
  return m ? static_cast<int>(__umulhi(static_cast<unsigned>(k), m)) : k;
}

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

// Window of the box, fitting when it holds at most cap cells.  Call after a
// barrier that follows all box_add_range calls.
__device__ __forceinline__ Window box_window(const BoxShared& b, int cap) {
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
  w.fits = !empty && vol <= cap;
  w.vol = w.fits ? static_cast<int>(vol) : 0;
  w.mz = w.fits ? div_magic(w.w[2]) : 0;
  w.my = w.fits ? div_magic(w.w[1]) : 0;
  return w;
}

// Window-local index of unwrapped cell c.
__device__ __forceinline__ int win_index(const Window& w, int cx, int cy, int cz) {
  return ((cx - w.o[0]) * w.w[1] + (cy - w.o[1])) * w.w[2] + (cz - w.o[2]);
}

// Physical (wrapped) mesh index of window cell number k (meshes have at
// most 2^30 cells, so 32 bits hold it).
__device__ __forceinline__ unsigned win_cell(const Window& w, int k, int mask, int lm) {
  const int t = div_by(k, w.mz);
  const int u = div_by(t, w.my);
  const unsigned cz = static_cast<unsigned>(w.o[2] + (k - t * w.w[2])) & mask;
  const unsigned cy = static_cast<unsigned>(w.o[1] + (t - u * w.w[1])) & mask;
  const unsigned cx = static_cast<unsigned>(w.o[0] + u) & mask;
  return (cx << (2 * lm)) | (cy << lm) | cz;
}

// Source pointers of NF mesh fields read through one window.
template <typename T, int NF>
struct Fields {
  const T* p[NF];
};

// Loads NF fields of the window into lds[f * kGCap + k].  Each thread issues
// the loads of kBatch cells (all fields) before storing any of them, so the
// loads of a batch are in flight together instead of one at a time.
constexpr int kBatch = 8;

template <typename T, int NF>
__device__ __forceinline__ void win_load(const Window& w, const Fields<T, NF>& src, int lm,
                                         T* lds) {
  const int mask = (1 << lm) - 1;
  for (int base = 0; base < w.vol; base += kBatch * kThreads) {
    T v[kBatch][NF];
    // Cells past the window end load the last window cell (in bounds) and
    // are not stored, so the loads need no branches and stay in flight
    // together.
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = min(base + j * kThreads + static_cast<int>(threadIdx.x), w.vol - 1);
      const unsigned c = win_cell(w, k, mask, lm);
#pragma unroll
      for (int f = 0; f < NF; ++f) v[j][f] = src.p[f][c];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = base + j * kThreads + threadIdx.x;
      if (k < w.vol) {
#pragma unroll
        for (int f = 0; f < NF; ++f) lds[f * kGCap + k] = v[j][f];
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
    unsigned c[kBatch];
    // Reads past the window end are clamped to its last cell and dropped.
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = min(base + j * kThreads + static_cast<int>(threadIdx.x), w.vol - 1);
      c[j] = win_cell(w, k, mask, lm);
      v[j] = static_cast<T>(acc[k]);
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = base + j * kThreads + threadIdx.x;
      if (k < w.vol && v[j] != T(0)) pk::atomic_add(dst + c[j], v[j]);
    }
  }
}

// Window statistics while kernel timing is on, spread over kStatSlots
// groups of kStatWords counters (block b uses group b mod kStatSlots) so
// blocks do not queue on one address: [0] windows, [1] windows that did not
// fit (their tile took the direct path), [2] cells of the windows that fit,
// [3] largest window asked for, in cells.
constexpr int kStatSlots = 64;
constexpr int kStatWords = 4;

__device__ __forceinline__ void tile_stats(const Window& w, const BoxShared& b,
                                           unsigned long long* stats) {
  if (stats && threadIdx.x == 0) {
    unsigned long long* s = stats + kStatWords * (blockIdx.x % kStatSlots);
    long long vol = 1;
    for (int a = 0; a < 3; ++a) vol *= (long long)b.hi[a] - (long long)b.lo[a] + 1;
    atomicAdd(s, 1ull);
    if (!w.fits) atomicAdd(s + 1, 1ull);
    atomicAdd(s + 2, (unsigned long long)w.vol);
    atomicMax(s + 3, (unsigned long long)(vol > 0 ? vol : 0));
  }
}

}  // namespace tk
}  // namespace ic
