// Tiled particle kernels: the paint, fused kick-drift-paint, final kick +
// RSD + data paint, and adjoint kernels of particles.h, restructured around
// Lagrangian tiles with LDS mesh windows (tiles.h).  Each kernel computes the
// same per-particle arithmetic as its direct counterpart; only where mesh
// values are read from and accumulated into changes.
#pragma once

#include "tiles.h"

namespace ic {
namespace pk {

using tk::BoxShared;
using tk::kPer;
using tk::kThreads;
using tk::TileGeom;
using tk::Window;

// Per-thread particle slots of a tile.
template <typename T>
struct Slots {
  bool ok[kPer];
  long long n[kPer];
  int idx[kPer][3];
};

template <typename T>
__device__ __forceinline__ void load_slots(Slots<T>& sl, const TileGeom& tg, int lp) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) sl.ok[k] = tk::tile_particle(tg, lp, k, sl.idx[k], sl.n[k]);
}

// Paints weight w times value v of stencil s into the FP64 window (LDS
// atomics) or, for a window that does not fit, straight into the mesh.
template <typename T>
__device__ __forceinline__ void paint_stencil(const Stencil<T>& s, T v, const Window& w,
                                              tk::Acc* acc, int lm, T* __restrict__ mesh) {
  if (w.fits) {
    for_corners_xyz(s, [&](int cx, int cy, int cz, T wt, T, T, T) {
      atomicAdd(&acc[tk::win_index(w, cx, cy, cz)], tk::Acc(wt) * tk::Acc(v));
    });
  } else {
    for_corners(s, lm, [&](long long c, T wt, T, T, T) { atomic_add(mesh + c, wt * v); });
  }
}

// Zeroes the window, paints one value per selected slot, flushes the window.
// Every thread of the block calls it (it holds barriers).
template <typename T>
__device__ __forceinline__ void paint_pass(const Stencil<T> st[kPer], const bool ok[kPer],
                                           const T v[kPer], const Window& w, tk::Acc* acc,
                                           int lm, T* __restrict__ mesh) {
  if (w.fits) tk::win_zero(w, acc);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (ok[k]) paint_stencil<T>(st[k], v[k], w, acc, lm, mesh);
  __syncthreads();
  if (w.fits) tk::win_flush(w, acc, lm, mesh);
}

// F_f = sum over corners of W g_f, from the window or from the mesh.
template <typename T, int NF>
__device__ __forceinline__ void gather_stencil(const Stencil<T>& s, const Window& w, const T* lds,
                                               int lm, const tk::Fields<T, NF>& mesh,
                                               T out[NF]) {
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f] = T(0);
  if (w.fits) {
    for_corners_xyz(s, [&](int cx, int cy, int cz, T wt, T, T, T) {
      const int k = tk::win_index(w, cx, cy, cz);
#pragma unroll
      for (int f = 0; f < NF; ++f) out[f] += wt * lds[f * tk::kGCap + k];
    });
  } else {
    for_corners(s, lm, [&](long long c, T wt, T, T, T) {
#pragma unroll
      for (int f = 0; f < NF; ++f) out[f] += wt * mesh.p[f][c];
    });
  }
}

// Window of the stencils held in st[] (ok[] marks the slots to cover), of
// at most cap cells.
template <typename T>
__device__ __forceinline__ Window window_of(BoxShared& bs, const Stencil<T> st[kPer],
                                            const bool ok[kPer], int cap) {
  tk::box_init(bs);
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!ok[k]) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], st[k].i0[a]);
      hi[a] = max(hi[a], st[k].i0[a] + 1);
    }
  }
  __syncthreads();
  tk::box_add_range(bs, lo, hi);
  __syncthreads();
  Window w = tk::box_window(bs, cap);
  __syncthreads();
  return w;
}

// Runs body(window) once for the tile.  A tile whose window exceeds cap
// cells gets a window with fits == false, and body then takes the direct
// global path.  (Splitting such tiles into smaller windows inside a loop
// makes the compiler hoist the stencil weights out of the loop and doubles
// the register demand of every tiled kernel.)
template <typename T, class Body>
__device__ __forceinline__ void with_window(BoxShared& bs, const Stencil<T> st[kPer],
                                            const bool ok[kPer], int cap,
                                            unsigned long long* __restrict__ stats,
                                            Body&& body) {
  const Window w = window_of(bs, st, ok, cap);
  tk::tile_stats(w, bs, stats);
  body(w);
}

// rho(c) += sum_n W(q_n + d_n - c).
template <typename T>
__global__ __launch_bounds__(kThreads, tk::kWaves) void k_paint_t(
    const T* __restrict__ d, long long P, int lp, TileGeom tg, Grid<T> g, T* __restrict__ rho,
    unsigned long long* __restrict__ stats) {
  __shared__ tk::Acc acc[tk::kPCap];
  __shared__ BoxShared bs;
  Slots<T> sl;
  load_slots(sl, tg, lp);
  Stencil<T> st[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!sl.ok[k]) continue;
    T dsp[3];
    load3(d, P, sl.n[k], dsp);
    st[k] = stencil(sl.idx[k], g.ratio, dsp, g.inv_cell, g.cell);
  }
  T one[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) one[k] = T(1);
  with_window(bs, st, sl.ok, tk::kPCap, stats, [&](const Window& w) {
    paint_pass<T>(st, sl.ok, one, w, acc, g.lm, rho);
  });
}

// g_bar_j(c) += coef * sum_n v_nj W(q_n + d_n - c), three meshes M apart.
template <typename T>
__global__ __launch_bounds__(kThreads, tk::kWaves) void k_paint_vec_t(
    const T* __restrict__ d, const T* __restrict__ v, T coef, long long P, int lp, TileGeom tg,
    Grid<T> g, T* __restrict__ out, long long M, unsigned long long* __restrict__ stats) {
  __shared__ tk::Acc acc[tk::kPCap];
  __shared__ BoxShared bs;
  Slots<T> sl;
  load_slots(sl, tg, lp);
  Stencil<T> st[kPer];
  T vv[kPer][3] = {};
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!sl.ok[k]) continue;
    T dsp[3];
    load3(d, P, sl.n[k], dsp);
    load3(v, P, sl.n[k], vv[k]);
#pragma unroll
    for (int a = 0; a < 3; ++a) vv[k][a] *= coef;
    st[k] = stencil(sl.idx[k], g.ratio, dsp, g.inv_cell, g.cell);
  }
  with_window(bs, st, sl.ok, tk::kPCap, stats, [&](const Window& w) {
    // One field at a time through one FP64 window.
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
      if (f > 0) __syncthreads();  // the previous flush has read the window
      T vf[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) vf[k] = vv[k][f];
      paint_pass<T>(st, sl.ok, vf, w, acc, g.lm, out + f * M);
    }
  });
}

// Fused step: readout of g at d_cur, kick p += kick F; drift
// d_next = d_cur + drift p and paint rho at d_next.
template <typename T>
__global__ __launch_bounds__(kThreads, tk::kWaves) void k_pm_step_t(
    const T* __restrict__ dcur, T* __restrict__ p, const T* __restrict__ g, long long M, T kick,
    T drift, T* __restrict__ dnext, T* __restrict__ rho, long long P, int lp, TileGeom tg,
    Grid<T> gr, unsigned long long* __restrict__ stats) {
  __shared__ __align__(16) unsigned char smem[tk::lds_bytes<T>(3)];
  T* lds = reinterpret_cast<T*>(smem);
  tk::Acc* acc = reinterpret_cast<tk::Acc*>(smem);
  __shared__ BoxShared bs;
  Slots<T> sl;
  load_slots(sl, tg, lp);
  Stencil<T> st[kPer], st2[kPer];
  T dsp[kPer][3], mom[kPer][3];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!sl.ok[k]) continue;
    load3(dcur, P, sl.n[k], dsp[k]);
    load3(p, P, sl.n[k], mom[k]);
    st[k] = stencil(sl.idx[k], gr.ratio, dsp[k], gr.inv_cell, gr.cell);
  }
  const tk::Fields<T, 3> gf = {{g, g + M, g + 2 * M}};
  with_window(bs, st, sl.ok, tk::kGCap, stats, [&](const Window& w) {
    if (w.fits) tk::win_load<T, 3>(w, gf, gr.lm, lds);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!sl.ok[k]) continue;
      T F[3];
      gather_stencil<T, 3>(st[k], w, lds, gr.lm, gf, F);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        mom[k][a] += kick * F[a];
        p[a * P + sl.n[k]] = mom[k][a];
        dsp[k][a] += drift * mom[k][a];
        dnext[a * P + sl.n[k]] = dsp[k][a];
      }
      st2[k] = stencil(sl.idx[k], gr.ratio, dsp[k], gr.inv_cell, gr.cell);
    }
  });
  T one[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) one[k] = T(1);
  with_window(bs, st2, sl.ok, tk::kPCap, stats, [&](const Window& w) {
    paint_pass<T>(st2, sl.ok, one, w, acc, gr.lm, rho);
  });
}

// Last kick (readout of g at d), then RSD and the data-grid paint.
template <typename T>
__global__ __launch_bounds__(kThreads, tk::kWaves) void k_final_t(
    const T* __restrict__ d, T* __restrict__ p, const T* __restrict__ g, long long M, T kick,
    Grid<T> gm, Rsd<T> rsd, Grid<T> gd, T* __restrict__ rho_d, long long P, int lp,
    TileGeom tg, unsigned long long* __restrict__ stats) {
  __shared__ __align__(16) unsigned char smem[tk::lds_bytes<T>(3)];
  T* lds = reinterpret_cast<T*>(smem);
  tk::Acc* acc = reinterpret_cast<tk::Acc*>(smem);
  __shared__ BoxShared bs;
  Slots<T> sl;
  load_slots(sl, tg, lp);
  Stencil<T> st[kPer], st2[kPer];
  T dsp[kPer][3], mom[kPer][3];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!sl.ok[k]) continue;
    load3(d, P, sl.n[k], dsp[k]);
    load3(p, P, sl.n[k], mom[k]);
    st[k] = stencil(sl.idx[k], gm.ratio, dsp[k], gm.inv_cell, gm.cell);
  }
  const tk::Fields<T, 3> gf = {{g, g + M, g + 2 * M}};
  with_window(bs, st, sl.ok, tk::kGCap, stats, [&](const Window& w) {
    if (w.fits) tk::win_load<T, 3>(w, gf, gm.lm, lds);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!sl.ok[k]) continue;
      T F[3], ds[3];
      gather_stencil<T, 3>(st[k], w, lds, gm.lm, gf, F);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        mom[k][a] += kick * F[a];
        p[a * P + sl.n[k]] = mom[k][a];
      }
      rsd_shift(rsd, sl.idx[k], dsp[k], mom[k], ds);
      st2[k] = stencil(sl.idx[k], gd.ratio, ds, gd.inv_cell, gd.cell);
    }
  });
  T one[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) one[k] = T(1);
  with_window(bs, st2, sl.ok, tk::kPCap, stats, [&](const Window& w) {
    paint_pass<T>(st2, sl.ok, one, w, acc, gd.lm, rho_d);
  });
}

// Adjoint of RSD + data paint (see k_data_adjoint), data-grid window.
template <typename T>
__global__ __launch_bounds__(kThreads, tk::kWaves) void k_data_adjoint_t(
    const T* __restrict__ d, const T* __restrict__ p, Rsd<T> rsd, Grid<T> gd,
    const T* __restrict__ rho_bar, T* __restrict__ dbar, T* __restrict__ pbar, long long P,
    int lp, TileGeom tg, unsigned long long* __restrict__ stats) {
  __shared__ T lds[tk::kGCap];
  __shared__ BoxShared bs;
  Slots<T> sl;
  load_slots(sl, tg, lp);
  Stencil<T> st[kPer];
  T dsp[kPer][3], mom[kPer][3];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!sl.ok[k]) continue;
    T ds[3];
    load3(d, P, sl.n[k], dsp[k]);
    load3(p, P, sl.n[k], mom[k]);
    rsd_shift(rsd, sl.idx[k], dsp[k], mom[k], ds);
    st[k] = stencil(sl.idx[k], gd.ratio, ds, gd.inv_cell, gd.cell);
  }
  const tk::Fields<T, 1> rf = {{rho_bar}};
  with_window(bs, st, sl.ok, tk::kGCap, stats, [&](const Window& w) {
    if (w.fits) tk::win_load<T, 1>(w, rf, gd.lm, lds);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!sl.ok[k]) continue;
      T xb[3] = {0, 0, 0};
      auto acc = [&](T r, T d0, T d1, T d2) {
        xb[0] += d0 * r;
        xb[1] += d1 * r;
        xb[2] += d2 * r;
      };
      if (w.fits)
        for_corners_xyz(st[k], [&](int cx, int cy, int cz, T, T d0, T d1, T d2) {
          acc(lds[tk::win_index(w, cx, cy, cz)], d0, d1, d2);
        });
      else
        for_corners(st[k], gd.lm,
                    [&](long long c, T, T d0, T d1, T d2) { acc(rho_bar[c], d0, d1, d2); });
#pragma unroll
      for (int a = 0; a < 3; ++a) xb[a] *= gd.inv_cell;
      T db[3] = {xb[0], xb[1], xb[2]}, pb[3] = {0, 0, 0};
      rsd_transpose(rsd, sl.idx[k], dsp[k], mom[k], xb, db, pb);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        dbar[a * P + sl.n[k]] = db[a];
        pbar[a * P + sl.n[k]] = pb[a];
      }
    }
  });
}

// Position cotangent of one force evaluation (see k_force_adjoint), with
// g (three meshes) and rho_bar read from one four-field window.
template <typename T>
__global__ __launch_bounds__(kThreads, tk::kWaves) void k_force_adjoint_t(
    const T* __restrict__ d, T* __restrict__ pbar, T* __restrict__ dbar, T coef,
    const T* __restrict__ g, const T* __restrict__ rho_bar, long long M, T drift, long long P,
    int lp, TileGeom tg, Grid<T> gm, unsigned long long* __restrict__ stats) {
  __shared__ T lds[4 * tk::kGCap];
  __shared__ BoxShared bs;
  Slots<T> sl;
  load_slots(sl, tg, lp);
  Stencil<T> st[kPer];
  T pb[kPer][3], db[kPer][3];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!sl.ok[k]) continue;
    T dsp[3];
    load3(d, P, sl.n[k], dsp);
    // The cotangents are loaded now so their latency overlaps the window phase.
    load3(pbar, P, sl.n[k], pb[k]);
    load3(dbar, P, sl.n[k], db[k]);
    st[k] = stencil(sl.idx[k], gm.ratio, dsp, gm.inv_cell, gm.cell);
  }
  const tk::Fields<T, 4> f4 = {{g, g + M, g + 2 * M, rho_bar}};
  with_window(bs, st, sl.ok, tk::kGCap, stats, [&](const Window& w) {
    if (w.fits) tk::win_load<T, 4>(w, f4, gm.lm, lds);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (!sl.ok[k]) continue;
      const long long n = sl.n[k];
      const T v0 = coef * pb[k][0], v1 = coef * pb[k][1], v2 = coef * pb[k][2];
      T xb[3] = {0, 0, 0};
      auto acc = [&](T g0, T g1, T g2, T r, T d0, T d1, T d2) {
        const T h = v0 * g0 + v1 * g1 + v2 * g2 + r;
        xb[0] += d0 * h;
        xb[1] += d1 * h;
        xb[2] += d2 * h;
      };
      if (w.fits)
        for_corners_xyz(st[k], [&](int cx, int cy, int cz, T, T d0, T d1, T d2) {
          const int c = tk::win_index(w, cx, cy, cz);
          acc(lds[c], lds[tk::kGCap + c], lds[2 * tk::kGCap + c], lds[3 * tk::kGCap + c], d0, d1,
              d2);
        });
      else
        for_corners(st[k], gm.lm, [&](long long c, T, T d0, T d1, T d2) {
          acc(g[c], g[M + c], g[2 * M + c], rho_bar[c], d0, d1, d2);
        });
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        db[k][a] += xb[a] * gm.inv_cell;
        dbar[a * P + n] = db[k][a];
        if (drift != T(0)) pbar[a * P + n] = pb[k][a] + drift * db[k][a];
      }
    }
  });
}

}  // namespace pk
}  // namespace ic
