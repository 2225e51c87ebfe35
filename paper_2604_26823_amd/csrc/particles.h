// Particle building blocks shared by the block-ordered kernels (blocks.h)
// and the lightcone (lightcone.h): cloud-in-cell stencils and weights, the
// readout of the force meshes, and the redshift-space distortion with its
// transpose (gfx950).
//
// Particles are lattice points q_n = n dq plus a displacement d_n stored in
// structure-of-arrays form [3][P] in lattice order, so consecutive threads
// hold spatially adjacent particles and their CIC stencils touch adjacent
// cells (coalesced gathers, clustered atomics).  The cell index is split into
// the exact integer lattice part (n * ratio) and floor(d / cell), which keeps
// FP32 positions accurate to the displacement's own rounding.
#pragma once

#include <limits>

#include "common.h"

namespace ic {
namespace pk {

template <typename T>
struct Stencil {
  int i0[3];
  T t[3];
};

// Lattice coordinates of particle index n on a side-np lattice (np = 2^lp).
__device__ __forceinline__ void lattice(long long n, int lp, int idx[3]) {
  const int mask = (1 << lp) - 1;
  idx[2] = static_cast<int>(n & mask);
  idx[1] = static_cast<int>((n >> lp) & mask);
  idx[0] = static_cast<int>(n >> (2 * lp));
}

// CIC stencil of the particle at lattice index idx displaced by dsp.  The
// fractional position t = (d - f cell) / cell takes the remainder d - f cell
// with one fused multiply-add, which is exact when the cell size is a binary
// fraction (L / N with N a power of two), so t carries the rounding of d only
// and not the larger rounding of d / cell at |d| of many cells.
template <typename T>
__device__ __forceinline__ Stencil<T> stencil(const int idx[3], int ratio, const T dsp[3],
                                              T inv_cell, T cell) {
  Stencil<T> s;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T f = floor(dsp[a] * inv_cell);
    T r = fma(-f, cell, dsp[a]);
    if (r < T(0)) {
      f -= T(1);
      r += cell;
    } else if (r >= cell) {
      f += T(1);
      r -= cell;
    }
    T t = r * inv_cell;
    if (t >= T(1)) t = T(1) - T(0.5) * std::numeric_limits<T>::epsilon();
    s.i0[a] = idx[a] * ratio + static_cast<int>(f);
    s.t[a] = t;
  }
  return s;
}

__device__ __forceinline__ long long cell_index(const int c[3], int mask, int lm) {
  return ((long long)(c[0] & mask) << (2 * lm)) | ((long long)(c[1] & mask) << lm) |
         (long long)(c[2] & mask);
}

// Geometry of one grid the particles are painted to or read from.
template <typename T>
struct Grid {
  int lm;      // log2 of the grid side
  int ratio;   // grid cells per lattice spacing (1 or 2)
  T inv_cell;  // grid side / box
  T cell;      // box / grid side
};

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// Calls f(cx, cy, cz, w, dw0, dw1, dw2) for the 8 CIC corners with unwrapped
// cell coordinates, w the weight and dwa its derivative along axis a in
// units of 1/cell.
template <typename T, class F>
__device__ __forceinline__ void for_corners_xyz(const Stencil<T>& s, F&& f) {
#pragma unroll
  for (int ox = 0; ox < 2; ++ox) {
    const T wx = ox ? s.t[0] : T(1) - s.t[0];
    const T gx = ox ? T(1) : T(-1);
#pragma unroll
    for (int oy = 0; oy < 2; ++oy) {
      const T wy = oy ? s.t[1] : T(1) - s.t[1];
      const T gy = oy ? T(1) : T(-1);
#pragma unroll
      for (int oz = 0; oz < 2; ++oz) {
        const T wz = oz ? s.t[2] : T(1) - s.t[2];
        const T gz = oz ? T(1) : T(-1);
        f(s.i0[0] + ox, s.i0[1] + oy, s.i0[2] + oz, wx * wy * wz, gx * wy * wz, wx * gy * wz,
          wx * wy * gz);
      }
    }
  }
}

// Calls f(cell, w, dw0, dw1, dw2) for the 8 CIC corners, where w is the
// weight and dwa its derivative along axis a in units of 1/cell.
template <typename T, class F>
__device__ __forceinline__ void for_corners(const Stencil<T>& s, int lm, F&& f) {
  const int mask = (1 << lm) - 1;
#pragma unroll
  for (int ox = 0; ox < 2; ++ox) {
    const T wx = ox ? s.t[0] : T(1) - s.t[0];
    const T gx = ox ? T(1) : T(-1);
#pragma unroll
    for (int oy = 0; oy < 2; ++oy) {
      const T wy = oy ? s.t[1] : T(1) - s.t[1];
      const T gy = oy ? T(1) : T(-1);
#pragma unroll
      for (int oz = 0; oz < 2; ++oz) {
        const T wz = oz ? s.t[2] : T(1) - s.t[2];
        const T gz = oz ? T(1) : T(-1);
        const int c[3] = {s.i0[0] + ox, s.i0[1] + oy, s.i0[2] + oz};
        f(cell_index(c, mask, lm), wx * wy * wz, gx * wy * wz, wx * gy * wz, wx * wy * gz);
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void load3(const T* __restrict__ v, long long P, long long n, T out[3]) {
  out[0] = v[n];
  out[1] = v[P + n];
  out[2] = v[2 * P + n];
}

// Readout of the three force meshes at particle positions: F_j = sum W g_j.
template <typename T>
__device__ __forceinline__ void readout3(const Stencil<T>& s, int lm, const T* __restrict__ g,
                                         long long M, T F[3]) {
  F[0] = F[1] = F[2] = T(0);
  for_corners(s, lm, [&](long long c, T w, T, T, T) {
    F[0] += w * g[c];
    F[1] += w * g[M + c];
    F[2] += w * g[2 * M + c];
  });
}

// Redshift-space displacement.  mode 1: shift c p_z along z; mode 2: shift
// c (p . u) u with u the unit vector from the observer to the wrapped
// position; r = 0 gives no shift.
template <typename T>
struct Rsd {
  int mode;
  int n;  // lattice side
  T c;
  T box;
  T dq;
  T obs[3];
};

// Periodic image in [0, box) of the position idx * dq + d along one axis.
// Which image is taken is decided by comparing d with the exactly
// representable distances to the box faces, -idx dq and (n - idx) dq, rather
// than by rounding the sum first: the line of sight from a corner observer
// jumps at the faces, and this keeps FP32 on the same side as the exact
// position unless d itself is within its own rounding of a face.
template <typename T>
__device__ __forceinline__ T wrap_position(int idx, T d, const Rsd<T>& r) {
  const T lo = -static_cast<T>(idx) * r.dq;
  const T hi = static_cast<T>(r.n - idx) * r.dq;
  if (d >= lo && d < hi) return static_cast<T>(idx) * r.dq + d;
  if (d >= hi && d < hi + r.box) return static_cast<T>(idx - r.n) * r.dq + d;
  if (d < lo && d >= lo - r.box) return static_cast<T>(idx + r.n) * r.dq + d;
  const T x = static_cast<T>(idx) * r.dq + d;
  T y = x - r.box * floor(x / r.box);
  if (y < T(0)) y += r.box;
  if (y >= r.box) y -= r.box;
  return y;
}

template <typename T>
__device__ __forceinline__ void los(const Rsd<T>& r, const int idx[3], const T dsp[3], T u[3],
                                    T& dist) {
  T rr = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T y = wrap_position(idx[a], dsp[a], r);
    u[a] = y - r.obs[a];
    rr += u[a] * u[a];
  }
  dist = sqrt(rr);
  const T inv = dist > T(0) ? T(1) / dist : T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] *= inv;
}

template <typename T>
__device__ __forceinline__ void rsd_shift(const Rsd<T>& r, const int idx[3], const T dsp[3],
                                          const T mom[3], T out[3]) {
  out[0] = dsp[0];
  out[1] = dsp[1];
  out[2] = dsp[2];
  if (r.mode == 1) {
    out[2] += r.c * mom[2];
  } else if (r.mode == 2) {
    T u[3], dist;
    los(r, idx, dsp, u, dist);
    const T pu = r.c * (mom[0] * u[0] + mom[1] * u[1] + mom[2] * u[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] += pu * u[a];
  }
}

// Transpose of the RSD map at (d, p) applied to the redshift-space position
// cotangent xb: adds to db (which holds xb on entry) and sets pb.  Radial:
// with u the line of sight, P = I - u u^T and r the distance,
// db += (c / r) [(u.xb) P p + (p.u) P xb], pb = c (u.xb) u.
template <typename T>
__device__ __forceinline__ void rsd_transpose(const Rsd<T>& rsd, const int idx[3], const T dsp[3],
                                              const T mom[3], const T xb[3], T db[3], T pb[3]) {
  if (rsd.mode == 1) {
    pb[2] = rsd.c * xb[2];
  } else if (rsd.mode == 2) {
    T u[3], dist;
    los(rsd, idx, dsp, u, dist);
    const T ux = u[0] * xb[0] + u[1] * xb[1] + u[2] * xb[2];
    const T up = u[0] * mom[0] + u[1] * mom[1] + u[2] * mom[2];
    const T cr = dist > T(0) ? rsd.c / dist : T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T perp_p = mom[a] - up * u[a];
      const T perp_x = xb[a] - ux * u[a];
      db[a] += cr * (ux * perp_p + up * perp_x);
      pb[a] = rsd.c * ux * u[a];
    }
  }
}

}  // namespace pk
}  // namespace ic
