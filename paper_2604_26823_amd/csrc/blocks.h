// Eulerian block ordering of the particles (gfx950).
//
// The grid is cut into 8^3-cell blocks.  Every particle belongs to the block
// of its CIC base cell (the wrapped floor cell of its position), so all eight
// corners of its stencil fall inside that block extended by one cell on the
// upper side: a fixed 9^3-cell window.  After each drift the particles are
// counting-sorted by block (per-block counts with wavefront- or workgroup-aggregated
// atomics, an exclusive scan, then a scatter of the ids alone, with the new
// order's map back to the old: the density paint reads the new positions
// through that map and stores them in the new order, the next step reads the
// momenta through it; states that must be complete in their order move
// positions and momenta too), and every paint and readout then runs over work
// items of at most 1024 particles of one block, with the block's window in
// LDS:
//   * paints accumulate in LDS windows (FP64 adds for FP64 grids, exact
//     64-bit fixed-point adds for FP32 grids, see WinAcc); a block's only
//     item stores its 8^3 own cells (the items of a block with several add
//     them atomically), its z halo into a one-value-per-eight-cells field
//     the consumer adds while reading, and its x/y halo into a staging
//     slot that a second pass adds along whole grid rows: global float
//     atomics are served past the XCD's L2 and were the paints' largest
//     cost;
//   * gathers read their mesh fields from a window loaded with coalesced
//     loads.
// Unlike windows around Lagrangian patches, these windows cannot overflow,
// however far particles have moved or however strongly they cluster: a dense
// block simply yields more work items.
//
// The order inside a block follows the atomic ranks, so it can differ from
// run to run; the results then differ only by FP64 summation order in the
// LDS windows before the single rounding to the mesh type, and by the order
// of the global atomics, which is unordered anyway.
//
// Slot a of a sorted state holds the particle with Lagrangian index ids[a];
// dest[a] gives its slot in the next order.  The adjoint kernels of order n
// read the cotangents left in order n + 1 through dest and write them in
// order n, so no pass of its own moves them between orders (one gather takes
// order 0 back to the lattice order).
#pragma once

#include <type_traits>

#include "particles.h"

namespace ic {
namespace bk {

using pk::Grid;
using pk::Stencil;

constexpr int kLB = 3;                 // log2 of the block side in cells
constexpr int kB = 1 << kLB;           // block side
constexpr int kW = kB + 1;             // window side
constexpr int kWin = kW * kW * kW;     // window cells (729)
constexpr int kThreads = 256;
constexpr int kPer = 4;                // particles per thread
constexpr int kChunk = kThreads * kPer;  // particles per work item

// Blocks of one grid of side 2^lm (lm >= 3).
struct Layout {
  int lm;   // log2 of the grid side
  int lnb;  // log2 of the blocks per side
};

inline Layout layout_for(int lm) { return Layout{lm, lm - kLB}; }
inline unsigned block_count(const Layout& L) { return 1u << (3 * L.lnb); }
// Upper bound of the work items of P particles: each non-empty block gives
// ceil(count / kChunk) <= count / kChunk + 1 items.
inline unsigned max_items(const Layout& L, long long P) {
  return static_cast<unsigned>((P + kChunk - 1) / kChunk) + block_count(L);
}
// Workgroups of an item kernel: the item bound plus the slack of the XCD
// dealing (item_of).
inline unsigned item_grid(const Layout& L, long long P) { return max_items(L, P) + 8; }

// Up to six field pointers of one state array set.
template <typename T>
struct Ptrs {
  const T* p[6];
};
template <typename T>
struct MPtrs {
  T* p[6];
};

// Block of the (wrapped) base cell of stencil s; wraps s.i0 in place.
template <typename T>
__device__ __forceinline__ unsigned block_of(Stencil<T>& s, const Layout& L) {
  const int mask = (1 << L.lm) - 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) s.i0[a] &= mask;
  return (static_cast<unsigned>(s.i0[0] >> kLB) << (2 * L.lnb)) |
         (static_cast<unsigned>(s.i0[1] >> kLB) << L.lnb) |
         static_cast<unsigned>(s.i0[2] >> kLB);
}

// Origin (cell coordinates) of block b.
__device__ __forceinline__ void block_origin(unsigned b, const Layout& L, int o[3]) {
  const unsigned m = (1u << L.lnb) - 1;
  o[0] = static_cast<int>(b >> (2 * L.lnb)) << kLB;
  o[1] = static_cast<int>((b >> L.lnb) & m) << kLB;
  o[2] = static_cast<int>(b & m) << kLB;
}

// Window index of unwrapped cell c relative to origin o (c - o in [0, 8]).
__device__ __forceinline__ int win_index(const int o[3], int cx, int cy, int cz) {
  return ((cx - o[0]) * kW + (cy - o[1])) * kW + (cz - o[2]);
}

// Mesh index of window cell k of the window at origin o.
__device__ __forceinline__ unsigned win_cell(const int o[3], int k, const Layout& L) {
  const unsigned mask = (1u << L.lm) - 1;
  const int kx = k / (kW * kW), r = k - kx * kW * kW;
  const int ky = r / kW, kz = r - ky * kW;
  return ((static_cast<unsigned>(o[0] + kx) & mask) << (2 * L.lm)) |
         ((static_cast<unsigned>(o[1] + ky) & mask) << L.lm) |
         (static_cast<unsigned>(o[2] + kz) & mask);
}

// Lanes of the wavefront grouped by key with ballots: each active lane gets
// its group's first lane (leader) and its offset within the group, and the
// leader also gets the group size (0 elsewhere).  Every lane of the wavefront
// must call it; inactive lanes pass active = false.
struct RankTicket {
  unsigned base;  // the leader's reservation (atomic result), valid in leaders
  int leader;
  unsigned off;
};

__device__ __forceinline__ RankTicket group_by_key(unsigned key, bool active, unsigned& size) {
  const int lane = static_cast<int>(threadIdx.x & 63);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long todo = __ballot(active);
  RankTicket t{0u, 0, 0u};
  size = 0;
  while (todo) {
    const int leader = __ffsll(static_cast<long long>(todo)) - 1;
    const unsigned k = static_cast<unsigned>(__shfl(static_cast<int>(key), leader, 64));
    const unsigned long long same = __ballot(active && key == k);
    if (lane == leader) size = static_cast<unsigned>(__popcll(same));
    if (active && key == k) {
      t.leader = leader;
      t.off = static_cast<unsigned>(__popcll(same & below));
    }
    todo &= ~same;
  }
  return t;
}

// Rank of this lane's particle within its block: each group's leader adds
// the group size to the block count, all groups in the same atomic
// instruction (one round trip whatever the number of distinct keys), and the
// lanes of a group take consecutive ranks from the leader's result.
// Inactive lanes get 0.
__device__ __forceinline__ unsigned rank_in_block(unsigned key, bool active,
                                                  unsigned* __restrict__ count) {
  unsigned size;
  RankTicket t = group_by_key(key, active, size);
  if (size) t.base = atomicAdd(count + key, size);
  const unsigned base = static_cast<unsigned>(__shfl(static_cast<int>(t.base), t.leader, 64));
  return active ? base + t.off : 0u;
}

// Ranks aggregated over a workgroup whose particles all start in block b0:
// after a drift nearly every particle is in b0 or one of its 26 neighbours,
// so the wavefront groups reserve offsets on 27 LDS counters, one thread per
// non-empty counter then reserves the workgroup's range in that block's
// global count with one atomic, and each particle's rank is that base plus
// its offset.  Keys farther away keep the per-wavefront global atomic.
constexpr int kNbr = 27;

// Neighbour slot (0..26) of block key relative to block b0, or kNbr if the
// blocks are not adjacent (periodic block grid of side 2^lnb).
__device__ __forceinline__ int neighbour_slot(unsigned b0, unsigned key, const Layout& L) {
  const unsigned m = (1u << L.lnb) - 1;
  int slot = 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int sh = (2 - ax) * L.lnb;
    const unsigned d = ((key >> sh) - (b0 >> sh)) & m;
    int dd;
    if (d <= 1u) dd = static_cast<int>(d);
    else if (d == m) dd = -1;
    else return kNbr;
    slot = slot * 3 + dd + 1;
  }
  return slot;
}

// Block key of neighbour slot s of block b0.
__device__ __forceinline__ unsigned neighbour_key(unsigned b0, int s, const Layout& L) {
  const unsigned m = (1u << L.lnb) - 1;
  const int dd[3] = {s / 9 - 1, (s / 3) % 3 - 1, s % 3 - 1};
  unsigned key = 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int sh = (2 - ax) * L.lnb;
    key |= ((((b0 >> sh) & m) + static_cast<unsigned>(dd[ax])) & m) << sh;
  }
  return key;
}

// First half: each wavefront group's leader reserves the group's offsets,
// on the workgroup counter wcnt[slot] for neighbour keys, else on the global
// count; all of a thread's reservations can be in flight at once.
__device__ __forceinline__ RankTicket rank_issue_wg(unsigned key, int slot, bool active,
                                                    unsigned* __restrict__ count,
                                                    unsigned* wcnt) {
  unsigned size;
  RankTicket t = group_by_key(key, active, size);
  if (size) t.base = slot < kNbr ? atomicAdd(wcnt + slot, size) : atomicAdd(count + key, size);
  return t;
}

// Between the halves (with barriers around it): the workgroup's ranges.
__device__ __forceinline__ void rank_reserve_wg(unsigned b0, const Layout& L,
                                                unsigned* __restrict__ count, const unsigned* wcnt,
                                                unsigned* wbase) {
  const int t = static_cast<int>(threadIdx.x);
  if (t < kNbr && wcnt[t]) wbase[t] = atomicAdd(count + neighbour_key(b0, t, L), wcnt[t]);
}

__device__ __forceinline__ unsigned rank_finish_wg(const RankTicket& t, int slot, bool active,
                                                   const unsigned* wbase) {
  unsigned base = static_cast<unsigned>(__shfl(static_cast<int>(t.base), t.leader, 64));
  if (slot < kNbr) base += wbase[slot];
  return active ? base + t.off : 0u;
}

// ---------------------------------------------------------------- sorting
// Key and rank of every slot: the block of the stencil of displacement d
// (particle ids[a], or a when ids is null) on grid g.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_keys(const T* __restrict__ d,
                                                   const unsigned* __restrict__ ids, long long P,
                                                   int lp, Grid<T> g, Layout L,
                                                   unsigned* __restrict__ count,
                                                   unsigned* __restrict__ key,
                                                   unsigned* __restrict__ rank) {
  const long long a = blockIdx.x * (long long)kThreads + threadIdx.x;
  const bool ok = a < P;
  unsigned b = 0;
  if (ok) {
    const long long j = ids ? static_cast<long long>(ids[a]) : a;
    int idx[3];
    pk::lattice(j, lp, idx);
    T dsp[3];
    pk::load3(d, P, a, dsp);
    Stencil<T> s = pk::stencil(idx, g.ratio, dsp, g.inv_cell, g.cell);
    b = block_of(s, L);
  }
  const unsigned r = rank_in_block(b, ok, count);
  if (ok) {
    key[a] = b;
    rank[a] = r;
  }
}

// Exclusive scan of the per-block counts and item counts
// (ceil(count / kChunk)) in three phases: chunk sums, a one-workgroup scan
// of the chunk sums, and the chunk-local scans with their offsets.  start and
// istart get nb + 1 entries (the last = the totals).
constexpr int kScanChunk = 2048;  // blocks per chunk (256 threads x 8)

static __global__ __launch_bounds__(256) void k_scan_sums(const unsigned* __restrict__ count,
                                                   unsigned nb, uint2* __restrict__ sums) {
  __shared__ unsigned sc[256], si[256];
  unsigned c = 0, it = 0;
  const unsigned base = blockIdx.x * kScanChunk;
  for (int j = 0; j < kScanChunk / 256; ++j) {
    const unsigned i = base + j * 256 + threadIdx.x;
    if (i < nb) {
      const unsigned v = count[i];
      c += v;
      it += (v + kChunk - 1) / kChunk;
    }
  }
  sc[threadIdx.x] = c;
  si[threadIdx.x] = it;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sc[threadIdx.x] += sc[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = make_uint2(sc[0], si[0]);
}

// In-place exclusive scan of n <= 1024 pairs by one workgroup of 1024 threads.
static __global__ __launch_bounds__(1024) void k_scan_top(uint2* __restrict__ sums, unsigned n) {
  __shared__ unsigned a[1024], b[1024];
  const unsigned t = threadIdx.x;
  const uint2 v = t < n ? sums[t] : make_uint2(0u, 0u);
  a[t] = v.x;
  b[t] = v.y;
  __syncthreads();
  for (unsigned off = 1; off < 1024; off <<= 1) {
    const unsigned xa = t >= off ? a[t - off] : 0u, xb = t >= off ? b[t - off] : 0u;
    __syncthreads();
    a[t] += xa;
    b[t] += xb;
    __syncthreads();
  }
  if (t < n) sums[t] = make_uint2(a[t] - v.x, b[t] - v.y);
}

static __global__ __launch_bounds__(256) void k_scan_out(const unsigned* __restrict__ count, unsigned nb,
                                                  const uint2* __restrict__ sums,
                                                  unsigned* __restrict__ start,
                                                  unsigned* __restrict__ istart) {
  __shared__ unsigned sc[256], si[256];
  constexpr int kPerT = kScanChunk / 256;
  const unsigned base = blockIdx.x * kScanChunk + threadIdx.x * kPerT;
  unsigned c[kPerT], it[kPerT], tc = 0, ti = 0;
#pragma unroll
  for (int j = 0; j < kPerT; ++j) {
    const unsigned i = base + j;
    const unsigned v = i < nb ? count[i] : 0u;
    c[j] = v;
    it[j] = (v + kChunk - 1) / kChunk;
    tc += c[j];
    ti += it[j];
  }
  sc[threadIdx.x] = tc;
  si[threadIdx.x] = ti;
  __syncthreads();
  for (unsigned off = 1; off < 256; off <<= 1) {
    const unsigned xa = threadIdx.x >= off ? sc[threadIdx.x - off] : 0u;
    const unsigned xb = threadIdx.x >= off ? si[threadIdx.x - off] : 0u;
    __syncthreads();
    sc[threadIdx.x] += xa;
    si[threadIdx.x] += xb;
    __syncthreads();
  }
  unsigned oc = sums[blockIdx.x].x + sc[threadIdx.x] - tc;
  unsigned oi = sums[blockIdx.x].y + si[threadIdx.x] - ti;
#pragma unroll
  for (int j = 0; j < kPerT; ++j) {
    const unsigned i = base + j;
    if (i < nb) {
      start[i] = oc;
      istart[i] = oi;
    }
    oc += c[j];
    oi += it[j];
    if (i + 1 == nb) {
      start[nb] = oc;
      istart[nb] = oi;
    }
  }
}

// Work items: item istart[b] + j = (block b, first slot start[b] + j kChunk).
static __global__ __launch_bounds__(256) void k_fill_items(const unsigned* __restrict__ start,
                                                    const unsigned* __restrict__ istart,
                                                    unsigned nb, uint2* __restrict__ items) {
  for (unsigned b = blockIdx.x * 256 + threadIdx.x; b < nb; b += gridDim.x * 256) {
    const unsigned s0 = start[b], s1 = start[b + 1];
    unsigned i = istart[b];
    for (unsigned s = s0; s < s1; s += kChunk) items[i++] = make_uint2(b, s);
  }
}

// Moves nf fields (and the ids) of slot a to slot start[key[a]] + rank[a] of
// the new order; dest[a] receives that slot.  ids_src null means identity.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter(
    const unsigned* __restrict__ key, const unsigned* __restrict__ rank,
    const unsigned* __restrict__ start, Ptrs<T> src, MPtrs<T> dst, int nf,
    const unsigned* __restrict__ ids_src, unsigned* __restrict__ ids_dst,
    unsigned* __restrict__ dest, long long P) {
  const long long a = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (a >= P) return;
  const unsigned s = start[key[a]] + rank[a];
  for (int f = 0; f < nf; ++f) dst.p[f][s] = src.p[f][a];
  ids_dst[s] = ids_src ? ids_src[a] : static_cast<unsigned>(a);
  dest[a] = s;
}

// The ids of slot a (a itself when ids_src is null) to slot
// s = start[key[a]] + rank[a] of the new order, dest[a] = s, and inv[s] = a:
// the new order's map back to this one, through which the next kernels read
// the state left in this order.
static __global__ __launch_bounds__(kThreads) void k_scatter_ids(
    const unsigned* __restrict__ key, const unsigned* __restrict__ rank,
    const unsigned* __restrict__ start, const unsigned* __restrict__ ids_src,
    unsigned* __restrict__ ids_dst, unsigned* __restrict__ dest, unsigned* __restrict__ inv,
    long long P) {
  const long long a = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (a >= P) return;
  const unsigned id = ids_src ? ids_src[a] : static_cast<unsigned>(a);
  const unsigned s = start[key[a]] + rank[a];
  ids_dst[s] = id;
  inv[s] = static_cast<unsigned>(a);
  dest[a] = s;
}

// dst_f[a] = src_f[dest[a]] for nf fields: values of the next order brought
// back to this one.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_back(const unsigned* __restrict__ dest,
                                                          Ptrs<T> src, MPtrs<T> dst, int nf,
                                                          long long P) {
  const long long a = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (a >= P) return;
  const unsigned s = dest[a];
  for (int f = 0; f < nf; ++f) dst.p[f][a] = src.p[f][s];
}

// dst_f[ids[a]] = src_f[a]: a sorted state back to lattice order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_to_lattice(const unsigned* __restrict__ ids,
                                                         Ptrs<T> src, MPtrs<T> dst, int nf,
                                                         long long P) {
  const long long a = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (a >= P) return;
  const unsigned j = ids[a];
  for (int f = 0; f < nf; ++f) dst.p[f][j] = src.p[f][a];
}

// ------------------------------------------------------------ work items
struct Items {
  const uint2* items;
  const unsigned* start;   // nb + 1 entries
  const unsigned* nitems;  // device pointer to the item total
  const unsigned* ids;
};

// Block, origin and slot range of this workgroup's item; false (for the
// whole workgroup) past the last item.  Workgroups are dealt to the eight
// XCDs round-robin (workgroup w runs on XCD w mod 8).  Gathers (CONTIG) take
// item (w mod 8) per + w / 8 with per = ceil(items / 8), so each XCD walks
// one contiguous range of neighbouring blocks whose windows share cache
// lines in that XCD's L2; paints take item w, so neighbouring blocks, whose
// flushes add into the same halo cells, run on different XCDs and their
// atomics do not queue behind each other.  The grid must hold at least
// items + 7 workgroups.
constexpr int kXcds = 8;

struct Item {
  unsigned b;
  int o[3];
  unsigned s0, s1;
  unsigned i;       // item index
  bool single;      // the block's only item (it holds at most kChunk particles)
};

template <bool CONTIG>
__device__ __forceinline__ bool item_of(const Items& it, const Layout& L, Item& m) {
  const unsigned n = *it.nitems;
  const unsigned w = blockIdx.x;
  unsigned i = w;
  if (CONTIG) {
    const unsigned per = (n + kXcds - 1) / kXcds;
    i = (w % kXcds) * per + w / kXcds;
    if (w / kXcds >= per) return false;
  }
  if (i >= n) return false;
  const uint2 v = it.items[i];
  m.b = v.x;
  m.s0 = v.y;
  const unsigned e = it.start[v.x + 1];
  m.s1 = (m.s0 + kChunk < e) ? m.s0 + kChunk : e;
  m.i = i;
  m.single = e - it.start[v.x] <= static_cast<unsigned>(kChunk);
  block_origin(m.b, L, m.o);
  return true;
}

// Slots a[k] = s0 + threadIdx.x + k kThreads of this thread in the item and
// whether they hold a particle; slots past the item's end are clamped to its
// first slot (an item is never empty).  The kernels issue the loads of all
// kPer particles from these slots in one branch-free run and wait once:
// behind a branch per particle, the in-order memory counter made every
// particle's loads wait for all of the previous particle's.
__device__ __forceinline__ void item_slots(const Item& m, long long (&a)[kPer],
                                           bool (&ok)[kPer]) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const long long s = static_cast<long long>(m.s0) + threadIdx.x + k * kThreads;
    ok[k] = s < static_cast<long long>(m.s1);
    a[k] = ok[k] ? s : static_cast<long long>(m.s0);
  }
}

// u[k] = map[a[k]] (particle ids, slot maps).
__device__ __forceinline__ void load_u32(const unsigned* __restrict__ map,
                                         const long long (&a)[kPer], unsigned (&u)[kPer]) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) u[k] = map[a[k]];
}

// v[k] = the three fields of f (P apart) at slot s[k].
template <typename T, typename S>
__device__ __forceinline__ void load3_at(const T* __restrict__ f, long long P,
                                         const S (&s)[kPer], T (&v)[kPer][3]) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) pk::load3(f, P, static_cast<long long>(s[k]), v[k]);
}

// Lagrangian lattice indices of the particle ids.
__device__ __forceinline__ void lattice_all(const unsigned (&id)[kPer], int lp,
                                            int (&idx)[kPer][3]) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) pk::lattice(static_cast<long long>(id[k]), lp, idx[k]);
}

template <typename T>
__device__ __forceinline__ Stencil<T> wrapped_stencil(const int idx[3], const T dsp[3],
                                                      const Grid<T>& g) {
  Stencil<T> s = pk::stencil(idx, g.ratio, dsp, g.inv_cell, g.cell);
  const int mask = (1 << g.lm) - 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) s.i0[a] &= mask;
  return s;
}

// Loads nf window fields (mesh fields src.p[f]) into lds[f * kWin + k].
template <typename T>
__device__ __forceinline__ void load_window(const int o[3], const Layout& L, const Ptrs<T>& src,
                                            int nf, T* lds) {
  constexpr int kIt = (kWin + kThreads - 1) / kThreads;
  T v[kIt][4];
#pragma unroll
  for (int j = 0; j < kIt; ++j) {
    const int k = min(static_cast<int>(threadIdx.x) + j * kThreads, kWin - 1);
    const unsigned c = win_cell(o, k, L);
#pragma unroll
    for (int f = 0; f < 4; ++f)
      if (f < nf) v[j][f] = src.p[f][c];
  }
#pragma unroll
  for (int j = 0; j < kIt; ++j) {
    const int k = static_cast<int>(threadIdx.x) + j * kThreads;
    if (k < kWin) {
#pragma unroll
      for (int f = 0; f < 4; ++f)
        if (f < nf) lds[f * kWin + k] = v[j][f];
    }
  }
}

// LDS accumulation of the paint windows.  FP64 grids: FP64 adds
// (ds_add_f64).  FP32 grids: 64-bit fixed point, value = integer x 2^-e
// (ds_add_u64 takes about half the time of ds_add_f64 on scattered cells
// of gfx950, and integer adds are exact, so the window sums do not depend
// on the order of the atomics).  e is chosen per work item so that nothing
// overflows: every contribution is at most amax in magnitude (CIC weights
// are at most 1), a window cell receives at most kChunk of them, and
// amax 2^e < 2^52, so every partial sum stays below 2^62.  The rounding of
// a contribution, at most 2^-53 amax, is far below the FP32 result's.
template <typename T>
struct WinAcc {
  using Cell = double;
  struct Scale {
    double s, inv;
  };
  __device__ static Scale scale_for(double) { return Scale{1.0, 1.0}; }
  __device__ static void add(Cell* c, double v, const Scale&) { atomicAdd(c, v); }
  __device__ static double get(Cell c, const Scale&) { return c; }
};
struct FixAcc {
  using Cell = unsigned long long;
  struct Scale {
    double s, inv;
  };
  // 2^e with amax 2^e < 2^52 (amax < 2^k from frexp, e = 52 - k)
  __device__ static Scale scale_for(double amax) {
    if (!(amax > 0.0)) return Scale{1.0, 1.0};
    int k;
    frexp(amax, &k);
    return Scale{ldexp(1.0, 52 - k), ldexp(1.0, k - 52)};
  }
  // The scale of a deterministic paint, one for the whole paint: amax 2^e
  // 2^lpc < 2^62, so that a cell may receive one contribution from each of
  // the 2^lpc particles (a particle adds to a cell at most once) without
  // overflow; the rounding of a contribution is at most 2^(lpc - 62) amax.
  __device__ static Scale scale_det(double amax, int lpc) {
    if (!(amax > 0.0)) return Scale{1.0, 1.0};
    int k;
    frexp(amax, &k);
    return Scale{ldexp(1.0, 62 - lpc - k), ldexp(1.0, k + lpc - 62)};
  }
  __device__ static void add(Cell* c, double v, const Scale& sc) {
    atomicAdd(c, static_cast<unsigned long long>(__double2ll_rn(v * sc.s)));
  }
  __device__ static double get(Cell c, const Scale& sc) {
    return static_cast<double>(static_cast<long long>(c)) * sc.inv;
  }
};
template <>
struct WinAcc<float> : FixAcc {};

// Window accumulator of a paint: WinAcc<T>, or fixed point in deterministic
// mode (DET) for both precisions.
template <typename T, bool DET>
using PaintAcc = typename std::conditional<DET, FixAcc, WinAcc<T>>::type;

// Largest |contribution| a deterministic paint's scale is chosen for: the
// CIC weights (at most 1) times coef times the largest |v| (vmax, device;
// null for a density paint).  Computed the same way by the paint and by
// k_det_to_field.
template <typename T>
__device__ __forceinline__ double det_amax(const double* vmax, T coef) {
  return vmax ? fabs(static_cast<double>(coef * static_cast<T>(*vmax))) : 1.0;
}

template <typename C>
__device__ __forceinline__ void zero_window(C* acc, int nf) {
  for (int k = threadIdx.x; k < nf * kWin; k += kThreads) acc[k] = C(0);
}

// Largest |x| over the workgroup's threads (red: kThreads / 64 doubles of
// LDS; every thread gets the result after the barrier the caller places
// between the two halves).
__device__ __forceinline__ void wg_max_issue(double x, double* red) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
}
__device__ __forceinline__ double wg_max_finish(const double* red) {
  double x = red[0];
  for (int w = 1; w < kThreads / 64; ++w) x = fmax(x, red[w]);
  return x;
}

// The window's halo, its 217 cells with a coordinate 8, belongs to the
// blocks above.  The 64 cells above in z only (kx, ky < 8, kz = 8) land on
// the lowest z layer of the block above in z; the 153 with kx = 8 or ky = 8
// are numbered x face (81), then y face without it (72).
constexpr int kHaloXY = kW * kW + kB * kW;

__device__ __forceinline__ int halo_xy_index(int kx, int ky, int kz) {
  return kx == kB ? ky * kW + kz : kW * kW + kx * kW + kz;
}

// Flush of nf FP64 windows; the fields and zh are zero before the paint.
// * The block's own 8^3 cells: plain stores when this item is the block's
//   only one (no other item of the launch writes them), else global atomic
//   adds of the non-zero cells.
// * The z halo: into zh, one value per lowest-z-layer cell of every block
//   (zh[f][(bz << lm | x) << lm | y], a grid field of one value per eight
//   cells along z, laid out so that a block's 8 x 8 values form runs of 8),
//   stored or atomically added by the same rule; the consumer adds it to the
//   cell (x, y, 8 bz).
// * The x and y halos: into this item's slot of the halo staging
//   (nf x kHaloXY values), added into the cells by k_halo_rows.
// Single-item blocks thus flush without global atomics.
template <typename T>
__device__ __forceinline__ void flush_owned(const Item& m, const Layout& L,
                                            const typename WinAcc<T>::Cell* acc,
                                            const typename WinAcc<T>::Scale& sc, int nf,
                                            const MPtrs<T>& dst, T* __restrict__ zh,
                                            T* __restrict__ halo) {
  constexpr int kIt = (kWin + kThreads - 1) / kThreads;
  T* hs = halo + static_cast<size_t>(m.i) * nf * kHaloXY;
  const long long zplane = 1ll << (2 * L.lm + L.lnb);  // zh values per field (n^3 / 8)
  const unsigned bmask = (1u << L.lnb) - 1;
#pragma unroll
  for (int j = 0; j < kIt; ++j) {
    const int k = static_cast<int>(threadIdx.x) + j * kThreads;
    if (k >= kWin) continue;
    const int kx = k / (kW * kW), r = k - kx * kW * kW;
    const int ky = r / kW, kz = r - ky * kW;
    if (kx < kB && ky < kB) {
      T* out[4];
      long long c;
      if (kz < kB) {
        c = win_cell(m.o, k, L);
        for (int f = 0; f < nf; ++f) out[f] = dst.p[f];
      } else {
        const unsigned bz = ((static_cast<unsigned>(m.o[2]) >> kLB) + 1) & bmask;
        c = ((static_cast<long long>(bz) << L.lm | (m.o[0] + kx)) << L.lm) | (m.o[1] + ky);
        for (int f = 0; f < nf; ++f) out[f] = zh + f * zplane;
      }
      for (int f = 0; f < nf; ++f) {
        const T v = static_cast<T>(WinAcc<T>::get(acc[f * kWin + k], sc));
        if (m.single)
          out[f][c] = v;
        else if (v != T(0))
          pk::atomic_add(out[f] + c, v);
      }
    } else {
      const int h = halo_xy_index(kx, ky, kz);
      for (int f = 0; f < nf; ++f) hs[f * kHaloXY + h] = static_cast<T>(WinAcc<T>::get(acc[f * kWin + k], sc));
    }
  }
}

// Before a paint of one order: zeroes the own cells (nf fields) and the
// z-halo entries of every block that no single work item owns, i.e. blocks
// with no particles or with several items (whose items add atomically); a
// block's only item stores all of them itself.  One wavefront per block:
// lane (kx, ky) clears the eight cells of its z row and its z-halo entry.
// istart: the order's item starts per block (nb + 1).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero_unowned(const unsigned* __restrict__ istart,
                                                           Layout L, int nf, MPtrs<T> dst,
                                                           T* __restrict__ zh) {
  const long long t = blockIdx.x * (long long)kThreads + threadIdx.x;
  const long long b = t >> 6;
  if (b >= (1ll << (3 * L.lnb))) return;
  if (istart[b + 1] - istart[b] == 1u) return;
  const int lane = static_cast<int>(t & 63);
  int o[3];
  block_origin(static_cast<unsigned>(b), L, o);
  const long long cx = o[0] + (lane >> 3), cy = o[1] + (lane & 7);
  const long long row = ((cx << L.lm) | cy) << L.lm | o[2];
  const long long zplane = 1ll << (2 * L.lm + L.lnb);
  const unsigned bz = ((static_cast<unsigned>(o[2]) >> kLB) + 1) & ((1u << L.lnb) - 1);
  const long long zc = ((static_cast<long long>(bz) << L.lm | cx) << L.lm) | cy;
  for (int f = 0; f < nf; ++f) {
#pragma unroll
    for (int z = 0; z < kB; ++z) dst.p[f][row + z] = T(0);
    zh[f * zplane + zc] = T(0);
  }
}

// Output of a paint in deterministic mode: the integer fields det (nf fields
// of ncells), their z halo zh (nf x ncells / 8, laid out as a paint's z
// halo) and x/y halo staging halo (nf x kHaloXY per item), the device
// maximum |v| the scale is chosen for (null for a density paint) and lpc =
// log2 of the particle count.
struct DetOut {
  unsigned long long* det;
  unsigned long long* zh;
  unsigned long long* halo;
  const double* vmax;
  long long ncells;
  int lpc;
};

// Flush of a deterministic paint: flush_owned's scheme with the windows'
// integer sums themselves (one scale for the whole paint): a single item
// stores its block's own cells and z-halo entries, the items of blocks with
// several add theirs with 64-bit integer atomics (det and zh zeroed there
// before the paint), and every item leaves its x/y halo in its staging
// slot for k_halo_rows.  Integer adds commute, so the result depends neither
// on the order of the atomics nor on which particles share an item.
__device__ __forceinline__ void flush_det(const Item& m, const Layout& L, const FixAcc::Cell* acc,
                                          int nf, const DetOut& dt) {
  constexpr int kIt = (kWin + kThreads - 1) / kThreads;
  unsigned long long* hs = dt.halo + static_cast<size_t>(m.i) * nf * kHaloXY;
  const long long zplane = 1ll << (2 * L.lm + L.lnb);  // zh values per field (n^3 / 8)
  const unsigned bmask = (1u << L.lnb) - 1;
#pragma unroll
  for (int j = 0; j < kIt; ++j) {
    const int k = static_cast<int>(threadIdx.x) + j * kThreads;
    if (k >= kWin) continue;
    const int kx = k / (kW * kW), r = k - kx * kW * kW;
    const int ky = r / kW, kz = r - ky * kW;
    if (kx < kB && ky < kB) {
      unsigned long long* out;
      long long c, fstride;
      if (kz < kB) {
        c = win_cell(m.o, k, L);
        out = dt.det;
        fstride = dt.ncells;
      } else {
        const unsigned bz = ((static_cast<unsigned>(m.o[2]) >> kLB) + 1) & bmask;
        c = ((static_cast<long long>(bz) << L.lm | (m.o[0] + kx)) << L.lm) | (m.o[1] + ky);
        out = dt.zh;
        fstride = zplane;
      }
      for (int f = 0; f < nf; ++f) {
        const unsigned long long v = acc[f * kWin + k];
        if (m.single)
          out[f * fstride + c] = v;
        else if (v)
          atomicAdd(out + f * fstride + c, v);
      }
    } else {
      const int h = halo_xy_index(kx, ky, kz);
      for (int f = 0; f < nf; ++f) hs[f * kHaloXY + h] = acc[f * kWin + k];
    }
  }
}

// The fields of a deterministic paint: out_f[i] = (det_f[i] + the z-halo
// entry of cell i when its z is a multiple of 8) 2^-e with the paint's scale
// (vmax, coef, lpc as given to the paint); lm = log2 of the grid side.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_det_to_field(const unsigned long long* __restrict__ det,
                                                           const unsigned long long* __restrict__ zh,
                                                           int nf, long long ncells, int lm,
                                                           const double* __restrict__ vmax,
                                                           T coef, int lpc, MPtrs<T> out) {
  const double inv = FixAcc::scale_det(det_amax<T>(vmax, coef), lpc).inv;
  const long long zplane = ncells >> kLB;
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < ncells;
       i += (long long)gridDim.x * kThreads) {
    const long long zi = ((i & ((1ll << lm) - 1)) >> kLB << (2 * lm)) | (i >> lm);
    const bool zcell = (i & (kB - 1)) == 0;
    for (int f = 0; f < nf; ++f) {
      const unsigned long long z = zh[f * zplane + zi];
      const unsigned long long v = det[f * ncells + i] + (zcell ? z : 0ull);
      out.p[f][i] = static_cast<T>(static_cast<double>(static_cast<long long>(v)) * inv);
    }
  }
}

// Cells that receive x/y halo values: those with x or y on a block's lowest
// layer (x = 8 i: every y; y = 8 j: x not on such a layer).  They are
// visited block face by block face, one wavefront per face: 2 nb^3 faces
// (the x faces of all blocks, then their y faces), 64 cells (lanes) each.
__host__ __device__ __forceinline__ long long face_waves(const Layout& L) {
  return 2ll << (3 * L.lnb);
}

// After a paint of one order: every face cell gets the x and y halo values
// that the items of the blocks below it in x or y (with or without z) wrote
// for it.  A wavefront takes the face of one block: on an x face lane
// (ly, lz) is cell (8 b0, 8 b1 + ly, 8 b2 + lz), on a y face lane (lx, lz)
// is cell (8 b0 + lx, 8 b1, 8 b2 + lz) with lx = 0 idle (an x face cell).
// The main halo value of the face's 64 cells then sits in one contiguous
// run of the staging of one item, and the four wavefronts of a workgroup
// take neighbouring faces along z, so the mesh rows they update are
// 128-byte runs.  istart: the order's item starts per block (nb + 1).
template <typename T, int NF>
__global__ __launch_bounds__(kThreads) void k_halo_rows(const T* __restrict__ halo,
                                                        const unsigned* __restrict__ istart,
                                                        Layout L, MPtrs<T> dst) {
  const long long t = blockIdx.x * (long long)kThreads + threadIdx.x;
  const long long w = t >> 6;
  if (w >= face_waves(L)) return;
  const int lane = static_cast<int>(t & 63);
  const long long nb3 = 1ll << (3 * L.lnb);
  const bool yface = w >= nb3;
  const long long q = yface ? w - nb3 : w;
  const unsigned bm = (1u << L.lnb) - 1;
  const unsigned bb[3] = {static_cast<unsigned>(q >> (2 * L.lnb)),
                          static_cast<unsigned>(q >> L.lnb) & bm, static_cast<unsigned>(q) & bm};
  const int l[3] = {yface ? lane >> 3 : 0, yface ? 0 : lane >> 3, lane & 7};
  if (yface && l[0] == 0) return;
  // The six neighbour classes a = 2..7 = (ax ay az) as bits 2 1 0 with ax or
  // ay set: whether the lane's cell takes that class's halo, the
  // neighbour's item range and the halo entry.  The item ranges of all
  // classes, then the first items' values, are loaded in one branch-free
  // run each (clamped to item 0 and selected where unused); further items
  // (blocks with several) follow in a loop.
  constexpr int kA = 6;
  bool use[kA];
  int h[kA];
  unsigned i0[kA], i1[kA];
#pragma unroll
  for (int q = 0; q < kA; ++q) {
    const int a = q + 2;
    const int ax = (a >> 2) & 1, ay = (a >> 1) & 1, az = a & 1;
    use[q] = !((ax && l[0]) || (ay && l[1]) || (az && l[2]));
    const unsigned nbk = (((bb[0] - ax) & bm) << (2 * L.lnb)) | (((bb[1] - ay) & bm) << L.lnb) |
                         ((bb[2] - az) & bm);
    h[q] = halo_xy_index(ax ? kB : l[0], ay ? kB : l[1], az ? kB : l[2]);
    i0[q] = istart[nbk];
    i1[q] = istart[nbk + 1];
  }
  T v[kA][NF];
#pragma unroll
  for (int q = 0; q < kA; ++q) {
    use[q] = use[q] && i0[q] < i1[q];
    const T* hs = halo + static_cast<size_t>(use[q] ? i0[q] : 0u) * NF * kHaloXY + h[q];
#pragma unroll
    for (int f = 0; f < NF; ++f) v[q][f] = hs[f * kHaloXY];
  }
  T sum[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    sum[f] = T(0);
#pragma unroll
    for (int q = 0; q < kA; ++q) sum[f] += use[q] ? v[q][f] : T(0);
  }
#pragma unroll
  for (int q = 0; q < kA; ++q) {
    if (!use[q]) continue;
    for (unsigned i = i0[q] + 1; i < i1[q]; ++i) {
      const T* hs = halo + static_cast<size_t>(i) * NF * kHaloXY + h[q];
#pragma unroll
      for (int f = 0; f < NF; ++f) sum[f] += hs[f * kHaloXY];
    }
  }
  const long long cx = (static_cast<long long>(bb[0]) << kLB) | l[0];
  const long long cy = (static_cast<long long>(bb[1]) << kLB) | l[1];
  const long long cz = (static_cast<long long>(bb[2]) << kLB) | l[2];
  const long long c = (((cx << L.lm) | cy) << L.lm) | cz;
#pragma unroll
  for (int f = 0; f < NF; ++f) dst.p[f][c] += sum[f];
}

// cell (x, y, 8 bz) += zh[(bz, x, y)] for one field of side 2^lm (the
// consumers that read a paint's field directly).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_add_zh(T* __restrict__ rho, const T* __restrict__ zh,
                                                     int lm, long long nz) {
  const long long i = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (i >= nz) return;
  const long long xy = i & ((1ll << (2 * lm)) - 1), bz = i >> (2 * lm);
  rho[(xy << lm) | (bz << kLB)] += zh[i];
}

// rho(c) += sum_n W(q_n + d_n - c) over the items of one order.  The
// displacement of slot a is d[a], or d[gsrc[a]] when it was left in the
// previous order (gsrc: this order's slots to that order's); then dcopy
// receives it in this order.  DET: the deterministic mode's output (dt)
// instead of rho, zh and halo.
template <typename T, bool DET>
__global__ __launch_bounds__(kThreads) void k_paint_b(const T* __restrict__ d,
                                                      const unsigned* __restrict__ gsrc,
                                                      T* __restrict__ dcopy, long long P,
                                                      int lp, Grid<T> g, Layout L, Items it,
                                                      T* __restrict__ rho, T* __restrict__ zh,
                                                      T* __restrict__ halo, DetOut dt) {
  using A = PaintAcc<T, DET>;
  __shared__ typename A::Cell acc[kWin];
  Item m;
  if (!item_of<false>(it, L, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned id[kPer];
  int idx[kPer][3];
  T dsp[kPer][3];
  item_slots(m, a, ok);  // loads in flight while the window is cleared
  load_u32(it.ids, a, id);
  if (gsrc) {
    unsigned sa[kPer];
    load_u32(gsrc, a, sa);
    load3_at(d, P, sa, dsp);
  } else {
    load3_at(d, P, a, dsp);
  }
  zero_window(acc, 1);
  if (dcopy) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!ok[k]) continue;
      dcopy[a[k]] = dsp[k][0];
      dcopy[P + a[k]] = dsp[k][1];
      dcopy[2 * P + a[k]] = dsp[k][2];
    }
  }
  lattice_all(id, lp, idx);
  typename A::Scale sc;  // weights are at most 1
  if constexpr (DET)
    sc = FixAcc::scale_det(1.0, dt.lpc);
  else
    sc = A::scale_for(1.0);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
    const Stencil<T> s = wrapped_stencil(idx[k], dsp[k], g);
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T w, T, T, T) {
      A::add(&acc[win_index(m.o, cx, cy, cz)], static_cast<double>(w), sc);
    });
  }
  __syncthreads();
  if constexpr (DET)
    flush_det(m, L, acc, 1, dt);
  else
    flush_owned<T>(m, L, acc, sc, 1, MPtrs<T>{{rho}}, zh, halo);
}

// g_bar_j(c) += coef * sum_n v_nj W(q_n + d_n - c), three meshes M apart; v
// of slot a is read at slot src[a] (the order the cotangents were left in).
// DET: the deterministic mode's output (dt, with dt.vmax = max |v|) instead
// of out, zh and halo.
template <typename T, bool DET>
__global__ __launch_bounds__(kThreads) void k_paint_vec_b(const T* __restrict__ d,
                                                          const T* __restrict__ v, T coef,
                                                          long long P, int lp, Grid<T> g,
                                                          Layout L, Items it, T* __restrict__ out,
                                                          long long M,
                                                          const unsigned* __restrict__ src,
                                                          T* __restrict__ zh,
                                                          T* __restrict__ halo, DetOut dt) {
  using A = PaintAcc<T, DET>;
  __shared__ typename A::Cell acc[3 * kWin];
  __shared__ double red[kThreads / 64];
  Item m;
  if (!item_of<false>(it, L, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned id[kPer], sa[kPer];
  int idx[kPer][3];
  T dsp[kPer][3], vv[kPer][3];
  item_slots(m, a, ok);  // loads in flight while the window is cleared
  load_u32(it.ids, a, id);
  load_u32(src, a, sa);
  load3_at(d, P, a, dsp);
  load3_at(v, P, sa, vv);
  zero_window(acc, 3);
  lattice_all(id, lp, idx);
  double amax = 0.0;  // largest |coef v| of the item (the weights are at most 1)
  if constexpr (!DET) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!ok[k]) continue;
#pragma unroll
      for (int q = 0; q < 3; ++q) amax = fmax(amax, fabs(static_cast<double>(coef * vv[k][q])));
    }
  }
  wg_max_issue(amax, red);
  __syncthreads();
  typename A::Scale sc;
  if constexpr (DET)
    sc = FixAcc::scale_det(det_amax<T>(dt.vmax, coef), dt.lpc);
  else
    sc = A::scale_for(wg_max_finish(red));
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
    const double v0 = static_cast<double>(coef * vv[k][0]),
                 v1 = static_cast<double>(coef * vv[k][1]),
                 v2 = static_cast<double>(coef * vv[k][2]);
    const Stencil<T> s = wrapped_stencil(idx[k], dsp[k], g);
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T w, T, T, T) {
      const int c = win_index(m.o, cx, cy, cz);
      const double wd = static_cast<double>(w);
      A::add(&acc[c], wd * v0, sc);
      A::add(&acc[kWin + c], wd * v1, sc);
      A::add(&acc[2 * kWin + c], wd * v2, sc);
    });
  }
  __syncthreads();
  if constexpr (DET)
    flush_det(m, L, acc, 3, dt);
  else
    flush_owned<T>(m, L, acc, sc, 3, MPtrs<T>{{out, out + M, out + 2 * M}}, zh, halo);
}

// Readout of g at d_n, kick p += kick F, drift d' = d_n + drift p; the new
// state goes to (dn, pn) in this order with its block key and rank on grid L
// (no keys when count is null: a replay into an order already recorded).
// The momentum of slot a is p[a], or p[pinv[a]] when the momenta were left
// in the previous order (pinv: this order's slots to that order's).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_step_b(
    const T* __restrict__ d, const T* __restrict__ p, const unsigned* __restrict__ pinv,
    const T* __restrict__ g, long long M, T kick, T drift, long long P, int lp, Grid<T> gr,
    Layout L, Items it, T* __restrict__ dn, T* __restrict__ pn, unsigned* __restrict__ count,
    unsigned* __restrict__ key, unsigned* __restrict__ rank) {
  __shared__ T lds[3 * kWin];
  Item m;
  if (!item_of<true>(it, L, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned b[kPer], id[kPer];
  int idx[kPer][3];
  T dsp[kPer][3], mom[kPer][3];
  item_slots(m, a, ok);  // particle loads in flight while the window loads
  load_u32(it.ids, a, id);
  if (pinv) {
    unsigned sa[kPer];
    load_u32(pinv, a, sa);
    load3_at(d, P, a, dsp);
    load3_at(p, P, sa, mom);
  } else {
    load3_at(d, P, a, dsp);
    load3_at(p, P, a, mom);
  }
  load_window<T>(m.o, L, Ptrs<T>{{g, g + M, g + 2 * M}}, 3, lds);
  lattice_all(id, lp, idx);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    b[k] = 0;
    if (!ok[k]) continue;
    T F[3] = {0, 0, 0};
    const Stencil<T> s = wrapped_stencil(idx[k], dsp[k], gr);
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T w, T, T, T) {
      const int c = win_index(m.o, cx, cy, cz);
      F[0] += w * lds[c];
      F[1] += w * lds[kWin + c];
      F[2] += w * lds[2 * kWin + c];
    });
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      mom[k][q] += kick * F[q];
      pn[q * P + a[k]] = mom[k][q];
      dsp[k][q] += drift * mom[k][q];
      dn[q * P + a[k]] = dsp[k][q];
    }
    Stencil<T> s2 = pk::stencil(idx[k], gr.ratio, dsp[k], gr.inv_cell, gr.cell);
    b[k] = block_of(s2, L);
  }
  if (!count) return;
  // ranks aggregated over the workgroup (see rank_issue_wg)
  __shared__ unsigned wcnt[kNbr], wbase[kNbr];
  if (threadIdx.x < kNbr) wcnt[threadIdx.x] = 0;
  __syncthreads();
  RankTicket t[kPer];
  int slot[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    slot[k] = neighbour_slot(m.b, b[k], L);
    t[k] = rank_issue_wg(b[k], slot[k], ok[k], count, wcnt);
  }
  __syncthreads();
  rank_reserve_wg(m.b, L, count, wcnt, wbase);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const unsigned r = rank_finish_wg(t[k], slot[k], ok[k], wbase);
    if (ok[k]) {
      key[a[k]] = b[k];
      rank[a[k]] = r;
    }
  }
}

// Position cotangent of one force evaluation with cotangent v = coef p_bar:
// d_bar += sum_c grad W(x - c) [sum_j v_j g_j(c) + rho_bar(c)], then the
// drift adjoint p_bar += drift d_bar; g (three meshes) and rho_bar are read
// from one four-field window.  p_bar and d_bar of slot a are read at slot
// src[a] of the order they were left in (the next order, or the data order)
// and the updates go to pbar_out[a] and dbar_out[a] in this order, so the
// move between orders costs no pass of its own.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_force_adjoint_b(
    const T* __restrict__ d, const T* __restrict__ pbar, const T* __restrict__ dbar, T coef,
    const T* __restrict__ g, const T* __restrict__ rho_bar, long long M, T drift, long long P,
    int lp, Grid<T> gm, Layout L, Items it, const unsigned* __restrict__ src,
    T* __restrict__ dbar_out, T* __restrict__ pbar_out) {
  __shared__ T lds[4 * kWin];
  Item m;
  if (!item_of<true>(it, L, m)) return;
  long long a[kPer];
  int idx[kPer][3];
  bool ok[kPer];
  unsigned id[kPer], sa[kPer];
  T dsp[kPer][3], pb[kPer][3], db[kPer][3];
  item_slots(m, a, ok);  // particle loads in flight while the window loads
  load_u32(it.ids, a, id);
  load_u32(src, a, sa);
  load3_at(d, P, a, dsp);
  load3_at(pbar, P, sa, pb);
  load3_at(dbar, P, sa, db);
  load_window<T>(m.o, L, Ptrs<T>{{g, g + M, g + 2 * M, rho_bar}}, 4, lds);
  lattice_all(id, lp, idx);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
    const Stencil<T> s = wrapped_stencil(idx[k], dsp[k], gm);
    const T v0 = coef * pb[k][0], v1 = coef * pb[k][1], v2 = coef * pb[k][2];
    T xb[3] = {0, 0, 0};
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T, T d0, T d1, T d2) {
      const int c = win_index(m.o, cx, cy, cz);
      const T h = v0 * lds[c] + v1 * lds[kWin + c] + v2 * lds[2 * kWin + c] + lds[3 * kWin + c];
      xb[0] += d0 * h;
      xb[1] += d1 * h;
      xb[2] += d2 * h;
    });
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      db[k][q] += xb[q] * gm.inv_cell;
      dbar_out[q * P + a[k]] = db[k][q];
      pbar_out[q * P + a[k]] = pb[k][q] + drift * db[k][q];
    }
  }
}

// Kick-synchronised snapshot of a state in its own block order (lightcone,
// section 2.2.1 item 3): snap = (d, p + half_kick F(d)), six fields P apart,
// F read out of the three force meshes g through the item's window.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_snapshot_b(
    const T* __restrict__ d, const T* __restrict__ p, const T* __restrict__ g, long long M,
    T half_kick, long long P, int lp, Grid<T> gm, Layout L, Items it, T* __restrict__ snap) {
  __shared__ T lds[3 * kWin];
  Item m;
  if (!item_of<true>(it, L, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned id[kPer];
  int idx[kPer][3];
  T dsp[kPer][3], mom[kPer][3];
  item_slots(m, a, ok);  // particle loads in flight while the window loads
  load_u32(it.ids, a, id);
  load3_at(d, P, a, dsp);
  load3_at(p, P, a, mom);
  load_window<T>(m.o, L, Ptrs<T>{{g, g + M, g + 2 * M}}, 3, lds);
  lattice_all(id, lp, idx);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
    T F[3] = {0, 0, 0};
    const Stencil<T> s = wrapped_stencil(idx[k], dsp[k], gm);
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T w, T, T, T) {
      const int c = win_index(m.o, cx, cy, cz);
      F[0] += w * lds[c];
      F[1] += w * lds[kWin + c];
      F[2] += w * lds[2 * kWin + c];
    });
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      snap[q * P + a[k]] = dsp[k][q];
      snap[(3 + q) * P + a[k]] = mom[k][q] + half_kick * F[q];
    }
  }
}

// Last kick (readout of g at d) of the momenta p into pout in this order,
// then the key and rank of the redshift-space position on the data grid
// (layout Ld).  The momentum of slot a is p[a] (pout may then be p: each
// slot is read and written by one thread), or p[pinv[a]] when the momenta
// were left in the previous order (pout apart from p).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_final_b(
    const T* __restrict__ d, const T* p, const unsigned* __restrict__ pinv, T* pout,
    const T* __restrict__ g, long long M, T kick, long long P, int lp, Grid<T> gm, Layout L,
    Items it, pk::Rsd<T> rsd, Grid<T> gd, Layout Ld, unsigned* __restrict__ count,
    unsigned* __restrict__ key, unsigned* __restrict__ rank) {
  __shared__ T lds[3 * kWin];
  Item m;
  if (!item_of<true>(it, L, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned b[kPer], id[kPer];
  int idx[kPer][3];
  T dsp[kPer][3], mom[kPer][3];
  item_slots(m, a, ok);  // particle loads in flight while the window loads
  load_u32(it.ids, a, id);
  if (pinv) {
    unsigned sa[kPer];
    load_u32(pinv, a, sa);
    load3_at(d, P, a, dsp);
    load3_at(p, P, sa, mom);
  } else {
    load3_at(d, P, a, dsp);
    load3_at(p, P, a, mom);
  }
  load_window<T>(m.o, L, Ptrs<T>{{g, g + M, g + 2 * M}}, 3, lds);
  lattice_all(id, lp, idx);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    b[k] = 0;
    if (!ok[k]) continue;
    T F[3] = {0, 0, 0}, ds[3];
    const Stencil<T> s = wrapped_stencil(idx[k], dsp[k], gm);
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T w, T, T, T) {
      const int c = win_index(m.o, cx, cy, cz);
      F[0] += w * lds[c];
      F[1] += w * lds[kWin + c];
      F[2] += w * lds[2 * kWin + c];
    });
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      mom[k][q] += kick * F[q];
      pout[q * P + a[k]] = mom[k][q];
    }
    pk::rsd_shift(rsd, idx[k], dsp[k], mom[k], ds);
    Stencil<T> s2 = pk::stencil(idx[k], gd.ratio, ds, gd.inv_cell, gd.cell);
    b[k] = block_of(s2, Ld);
  }
  // ranks aggregated over the workgroup around the data-grid block that
  // holds this mesh block's origin (see rank_issue_wg)
  const int rs = L.lm - Ld.lm;
  const unsigned b0 = ((static_cast<unsigned>(m.o[0] >> rs) >> kLB) << (2 * Ld.lnb)) |
                      ((static_cast<unsigned>(m.o[1] >> rs) >> kLB) << Ld.lnb) |
                      (static_cast<unsigned>(m.o[2] >> rs) >> kLB);
  __shared__ unsigned wcnt[kNbr], wbase[kNbr];
  if (threadIdx.x < kNbr) wcnt[threadIdx.x] = 0;
  __syncthreads();
  RankTicket t[kPer];
  int slot[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    slot[k] = neighbour_slot(b0, b[k], Ld);
    t[k] = rank_issue_wg(b[k], slot[k], ok[k], count, wcnt);
  }
  __syncthreads();
  rank_reserve_wg(b0, Ld, count, wcnt, wbase);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const unsigned r = rank_finish_wg(t[k], slot[k], ok[k], wbase);
    if (ok[k]) {
      key[a[k]] = b[k];
      rank[a[k]] = r;
    }
  }
}

// Data-grid paint of the redshift-space positions (items of the data order).
// DET: the deterministic mode's output (dt) instead of rho, zh and halo.
template <typename T, bool DET>
__global__ __launch_bounds__(kThreads) void k_data_paint_b(const T* __restrict__ d,
                                                           const T* __restrict__ p, long long P,
                                                           int lp, pk::Rsd<T> rsd, Grid<T> gd,
                                                           Layout Ld, Items it,
                                                           T* __restrict__ rho,
                                                           T* __restrict__ zh,
                                                           T* __restrict__ halo, DetOut dt) {
  using A = PaintAcc<T, DET>;
  __shared__ typename A::Cell acc[kWin];
  Item m;
  if (!item_of<false>(it, Ld, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned id[kPer];
  int idx[kPer][3];
  T dsp[kPer][3], mom[kPer][3];
  item_slots(m, a, ok);  // loads in flight while the window is cleared
  load_u32(it.ids, a, id);
  load3_at(d, P, a, dsp);
  load3_at(p, P, a, mom);
  zero_window(acc, 1);
  lattice_all(id, lp, idx);
  typename A::Scale sc;  // weights are at most 1
  if constexpr (DET)
    sc = FixAcc::scale_det(1.0, dt.lpc);
  else
    sc = A::scale_for(1.0);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
    T ds[3];
    pk::rsd_shift(rsd, idx[k], dsp[k], mom[k], ds);
    const Stencil<T> s = wrapped_stencil(idx[k], ds, gd);
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T w, T, T, T) {
      A::add(&acc[win_index(m.o, cx, cy, cz)], static_cast<double>(w), sc);
    });
  }
  __syncthreads();
  if constexpr (DET)
    flush_det(m, Ld, acc, 1, dt);
  else
    flush_owned<T>(m, Ld, acc, sc, 1, MPtrs<T>{{rho}}, zh, halo);
}

// Adjoint of the RSD + data paint (see pk::k_data_adjoint) over the data
// order: d_bar, p_bar in that order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_data_adjoint_b(
    const T* __restrict__ d, const T* __restrict__ p, long long P, int lp, pk::Rsd<T> rsd,
    Grid<T> gd, Layout Ld, Items it, const T* __restrict__ rho_bar, T* __restrict__ dbar,
    T* __restrict__ pbar) {
  __shared__ T lds[kWin];
  Item m;
  if (!item_of<true>(it, Ld, m)) return;
  long long a[kPer];
  bool ok[kPer];
  unsigned id[kPer];
  int idx[kPer][3];
  T dsp[kPer][3], mom[kPer][3];
  item_slots(m, a, ok);  // particle loads in flight while the window loads
  load_u32(it.ids, a, id);
  load3_at(d, P, a, dsp);
  load3_at(p, P, a, mom);
  load_window<T>(m.o, Ld, Ptrs<T>{{rho_bar}}, 1, lds);
  lattice_all(id, lp, idx);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
    T ds[3];
    pk::rsd_shift(rsd, idx[k], dsp[k], mom[k], ds);
    const Stencil<T> s = wrapped_stencil(idx[k], ds, gd);
    T xb[3] = {0, 0, 0};
    pk::for_corners_xyz(s, [&](int cx, int cy, int cz, T, T d0, T d1, T d2) {
      const T r = lds[win_index(m.o, cx, cy, cz)];
      xb[0] += d0 * r;
      xb[1] += d1 * r;
      xb[2] += d2 * r;
    });
#pragma unroll
    for (int q = 0; q < 3; ++q) xb[q] *= gd.inv_cell;
    T db[3] = {xb[0], xb[1], xb[2]}, pb[3] = {0, 0, 0};
    pk::rsd_transpose(rsd, idx[k], dsp[k], mom[k], xb, db, pb);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dbar[q * P + a[k]] = db[q];
      pbar[q * P + a[k]] = pb[q];
    }
  }
}

}  // namespace bk
}  // namespace ic
