// Lightcone of the particle output (paper section 2.2.1 item 3, appendix A).
//
// Snapshots of the kick-synchronised state are kept at interior steps, in
// the block order of their step (6 fields: displacement then momentum);
// following the recorded sort destinations from that order to the final one
// gives each final slot its slot in the snapshot (inverse maps built once per
// forward), so the gathers stay as spatially coherent as the orders are.  At the end of the
// forward model every particle's displacement and momentum are interpolated
// linearly in a between the snapshots that bracket a, and its crossing scale
// factor comes from the fixed point a <- A(|x(a) - observer|), started at
// a_final; A inverts the comoving distance and clamps to the snapshot range.
// The particle is then painted at x(a_i) with the RSD factor 1/(a_i^2 E(a_i)),
// carried as the momentum scaled by c(a_i)/c(a_final) so that the data paint
// and its adjoint stay those of the static model.  All scale-factor
// arithmetic is FP64; fields are in the working precision.
//
// The adjoint recomputes the fixed point per particle and runs it backwards:
// the cotangents of the final state go back in place (data order), those of
// the other snapshots to buffers in their snapshot's order, from which the
// reverse sweep injects them at their steps.
#pragma once

#include "particles.h"

namespace ic {
namespace lk {

constexpr int kMaxSnap = 4;
constexpr int kMaxIter = 16;
constexpr double kCOverH0 = 2997.92458;  // Mpc/h

// a(chi) as a cubic Hermite table on chi_k = chi_min + k h, k < n (values and
// slopes da/dchi); a_hi below chi_min, a_lo above chi_max.
struct LcTable {
  const double* a;
  const double* slope;
  double chi_min, chi_max, h, inv_h;
  int n;
  double a_lo, a_hi;
};

struct LcGeo {
  double a_snap[kMaxSnap];
  int J;           // snapshots, the last at a_final
  int iterations;
  double om;       // Omega_m of the flat cosmology
  double c_final;  // RSD factor at a_final
  LcTable tab;
};

__device__ __forceinline__ double hubble_E(double a, double om) {
  return sqrt(om / (a * a * a) + 1.0 - om);
}

// Crossing scale factor of comoving distance r; unc = r strictly inside
// the table (the derivative is zero where the result is clamped).
__device__ __forceinline__ double scale_factor(const LcTable& t, double r, bool& unc) {
  unc = r > t.chi_min && r < t.chi_max;
  if (r <= t.chi_min) return t.a_hi;
  if (r >= t.chi_max) return t.a_lo;
  const double u = (r - t.chi_min) * t.inv_h;
  const int k = min(static_cast<int>(u), t.n - 2);
  const double s = u - k, s1 = 1.0 - s;
  const double h00 = (1.0 + 2.0 * s) * s1 * s1, h10 = s * s1 * s1;
  const double h01 = s * s * (3.0 - 2.0 * s), h11 = s * s * (s - 1.0);
  return h00 * t.a[k] + h10 * t.h * t.slope[k] + h01 * t.a[k + 1] + h11 * t.h * t.slope[k + 1];
}

// The per-particle arrays below are indexed only by compile-time indices
// (NJ = the snapshot count, the fixed-point iterations unrolled up to KM >=
// iterations, KM = 4 or kMaxIter): a run-time index into them would put them
// in scratch memory.

// Bracket of a: lower snapshot j (the last with a_snap[j] <= a, at most
// NJ - 2), the weight t of snapshot j + 1 and the bracket's span in a.
template <int NJ>
__device__ __forceinline__ void bracket(const LcGeo& g, double a, int& j, double& t,
                                        double& span) {
  j = 0;
  double lo = g.a_snap[0], hi = g.a_snap[1];
#pragma unroll
  for (int i = 1; i < NJ - 1; ++i)
    if (g.a_snap[i] <= a) {
      j = i;
      lo = g.a_snap[i];
      hi = g.a_snap[i + 1];
    }
  span = hi - lo;
  t = (a - lo) / span;
}

// One particle's snapshot states (FP64 copies).
template <int NJ>
struct Snaps {
  double d[NJ][3];
  double p[NJ][3];
};

// Snapshot j of final slot a sits at slot inv[j P + a] of its own order.
template <typename T, int NJ>
__device__ __forceinline__ void load_snaps(const T* __restrict__ snap, const T* __restrict__ dS,
                                           const T* __restrict__ pS,
                                           const unsigned* __restrict__ inv, long long P,
                                           long long a, Snaps<NJ>& s) {
#pragma unroll
  for (int j = 0; j + 1 < NJ; ++j) {
    const T* b = snap + (long long)j * 6 * P;
    const long long sj = inv[(long long)j * P + a];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      s.d[j][q] = static_cast<double>(b[q * P + sj]);
      s.p[j][q] = static_cast<double>(b[(3 + q) * P + sj]);
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    s.d[NJ - 1][q] = static_cast<double>(dS[q * P + a]);
    s.p[NJ - 1][q] = static_cast<double>(pS[q * P + a]);
  }
}

// x[j] += (1 - t) v, x[j + 1] += t v for the bracket j of a run-time value
// (every x[i] is updated with a selected weight, so that no update is
// indexed by j).
template <int NJ>
__device__ __forceinline__ void add_bracket(double (&x)[NJ][3], int j, double t,
                                            const double v[3]) {
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const double w = (i == j ? 1.0 - t : 0.0) + (i == j + 1 ? t : 0.0);
#pragma unroll
    for (int q = 0; q < 3; ++q) x[i][q] += w * v[q];
  }
}

// Interpolated displacement (as T, the value the line of sight sees) and
// the slopes d x / d a, d p / d a of the bracket; j, t: the bracket.
template <typename T, int NJ>
__device__ __forceinline__ void interp(const LcGeo& g, const Snaps<NJ>& s, double a, T d[3],
                                       double p[3], double dd[3], double dp[3], int& j,
                                       double& t) {
  double span;
  bracket<NJ>(g, a, j, t, span);
  double d0[3], d1[3], p0[3], p1[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    d0[q] = s.d[0][q];
    d1[q] = s.d[1][q];
    p0[q] = s.p[0][q];
    p1[q] = s.p[1][q];
  }
#pragma unroll
  for (int i = 1; i + 1 < NJ; ++i)
    if (j == i) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        d0[q] = s.d[i][q];
        d1[q] = s.d[i + 1][q];
        p0[q] = s.p[i][q];
        p1[q] = s.p[i + 1][q];
      }
    }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    d[q] = static_cast<T>((1.0 - t) * d0[q] + t * d1[q]);
    p[q] = (1.0 - t) * p0[q] + t * p1[q];
    dd[q] = (d1[q] - d0[q]) / span;
    dp[q] = (p1[q] - p0[q]) / span;
  }
}

// Scale factors a^(0) = a_final, a^(k) = A(r(a^(k-1))), k <= iterations
// (<= KM); bit k of unc: a^(k) was not clamped.  Returns a^(iterations).
template <typename T, int NJ, int KM>
__device__ __forceinline__ double crossing(const LcGeo& g, const pk::Rsd<T>& rsd,
                                           const int idx[3], const Snaps<NJ>& s,
                                           double (&av)[KM + 1], unsigned& unc) {
  av[0] = g.a_snap[NJ - 1];
  unc = 0u;
  double last = av[0];
#pragma unroll
  for (int k = 1; k <= KM; ++k) {
    av[k] = last;
    if (k > g.iterations) continue;
    T d[3], u[3], dist;
    double p[3], dd[3], dp[3], t;
    int j;
    interp<T, NJ>(g, s, av[k - 1], d, p, dd, dp, j, t);
    pk::los(rsd, idx, d, u, dist);
    bool inside;
    av[k] = scale_factor(g.tab, static_cast<double>(dist), inside);
    if (inside) unc |= 1u << k;
    last = av[k];
  }
  return last;
}

// inv[dest_{m+k-1}( ... dest_m(a))] = a for the count orders that follow the
// snapshot's order m (dest: the first of count destination arrays, P apart):
// the snapshot slot of every final slot.
static __global__ __launch_bounds__(256) void k_snapshot_slots(const unsigned* __restrict__ dest,
                                                               int count,
                                                               unsigned* __restrict__ inv,
                                                               long long P) {
  for (long long a = blockIdx.x * (long long)blockDim.x + threadIdx.x; a < P;
       a += (long long)gridDim.x * blockDim.x) {
    long long x = a;
    for (int k = 0; k < count; ++k) x = dest[(long long)k * P + x];
    inv[x] = static_cast<unsigned>(a);
  }
}

// Lightcone state of every particle of the final order: displacement lcd,
// momentum scaled to the final RSD factor lcp, and the redshift-space
// displacement ds (for the data-grid keys).
template <typename T, int NJ, int KM>
__global__ __launch_bounds__(256) void k_lightcone(const T* __restrict__ dS, const T* __restrict__ pS,
                                                   const unsigned* __restrict__ ids,
                                                   const unsigned* __restrict__ inv,
                                                   const T* __restrict__ snap, LcGeo g,
                                                   pk::Rsd<T> rsd, T* __restrict__ lcd,
                                                   T* __restrict__ lcp, T* __restrict__ ds,
                                                   long long P, int lp) {
  for (long long a = blockIdx.x * (long long)blockDim.x + threadIdx.x; a < P;
       a += (long long)gridDim.x * blockDim.x) {
    int idx[3];
    pk::lattice(static_cast<long long>(ids[a]), lp, idx);
    Snaps<NJ> s;
    load_snaps<T, NJ>(snap, dS, pS, inv, P, a, s);
    double av[KM + 1];
    unsigned unc;
    const double ai = crossing<T, NJ, KM>(g, rsd, idx, s, av, unc);
    T d[3];
    double p[3], dd[3], dp[3], t;
    int j;
    interp<T, NJ>(g, s, ai, d, p, dd, dp, j, t);
    const double k = 1.0 / (ai * ai * hubble_E(ai, g.om) * g.c_final);
    T pe[3], out[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) pe[q] = static_cast<T>(k * p[q]);
    pk::rsd_shift(rsd, idx, d, pe, out);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      lcd[q * P + a] = d[q];
      lcp[q * P + a] = pe[q];
      ds[q * P + a] = out[q];
    }
  }
}

// Adjoint of k_lightcone.  dbar, pbar: cotangents of (lcd, lcp) in the data
// order on entry (slot dest[a] for final-order slot a), of the final state
// (d_S, p_S) on exit, in place; snapbar: cotangents of the other snapshots,
// each in its snapshot's order (every entry written).
template <typename T, int NJ, int KM>
__global__ __launch_bounds__(256) void k_lightcone_adjoint(
    const T* __restrict__ dS, const T* __restrict__ pS, const unsigned* __restrict__ ids,
    const unsigned* __restrict__ inv, const unsigned* __restrict__ dest,
    const T* __restrict__ snap, LcGeo g, pk::Rsd<T> rsd, T* __restrict__ dbar,
    T* __restrict__ pbar, T* __restrict__ snapbar, long long P, int lp) {
  for (long long a = blockIdx.x * (long long)blockDim.x + threadIdx.x; a < P;
       a += (long long)gridDim.x * blockDim.x) {
    const long long ad = dest[a];
    int idx[3];
    pk::lattice(static_cast<long long>(ids[a]), lp, idx);
    Snaps<NJ> s;
    load_snaps<T, NJ>(snap, dS, pS, inv, P, a, s);
    double av[KM + 1];
    unsigned unc;
    const double ai = crossing<T, NJ, KM>(g, rsd, idx, s, av, unc);
    double sd[NJ][3], sp[NJ][3];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) sd[j][q] = sp[j][q] = 0.0;
    const int K = g.iterations;
    T d[3];
    double p[3], dd[3], dp[3], t;
    int j;
    interp<T, NJ>(g, s, ai, d, p, dd, dp, j, t);
    // lcp = k(a) p with k = c(a) / c_final, c = 1 / (a^2 E)
    const double E = hubble_E(ai, g.om);
    const double k = 1.0 / (ai * ai * E * g.c_final);
    const double dlnE = -1.5 * g.om / (ai * ai * ai * ai * E * E);
    const double dk = -k * (2.0 / ai + dlnE);
    double xb[3], pb[3], abar = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      xb[q] = static_cast<double>(dbar[q * P + ad]);
      const double pe = static_cast<double>(pbar[q * P + ad]);
      pb[q] = k * pe;
      abar += dk * p[q] * pe + xb[q] * dd[q] + pb[q] * dp[q];
    }
    add_bracket<NJ>(sd, j, t, xb);
    add_bracket<NJ>(sp, j, t, pb);
#pragma unroll
    for (int it = KM; it >= 1; --it) {
      if (it > K) continue;
      const double ak = av[it];
      const double rbar = ((unc >> it) & 1u) ? abar * (-ak * ak * hubble_E(ak, g.om) / kCOverH0)
                                             : 0.0;
      T dk3[3], u[3], dist;
      double pk3[3], ddk[3], dpk[3];
      interp<T, NJ>(g, s, av[it - 1], dk3, pk3, ddk, dpk, j, t);
      pk::los(rsd, idx, dk3, u, dist);
      double rd[3];
      abar = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        rd[q] = rbar * static_cast<double>(u[q]);
        abar += rd[q] * ddk[q];
      }
      add_bracket<NJ>(sd, j, t, rd);
    }
#pragma unroll
    for (int jj = 0; jj + 1 < NJ; ++jj) {
      T* b = snapbar + (long long)jj * 6 * P;
      const long long sj = inv[(long long)jj * P + a];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        b[q * P + sj] = static_cast<T>(sd[jj][q]);
        b[(3 + q) * P + sj] = static_cast<T>(sp[jj][q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dbar[q * P + ad] = static_cast<T>(sd[NJ - 1][q]);
      pbar[q * P + ad] = static_cast<T>(sp[NJ - 1][q]);
    }
  }
}

// Launch of a lightcone kernel K<T, NJ, KM> for NJ = g.J snapshots (2 to 4)
// and KM = 4 when g.iterations <= 4 (the unrolled iterates stay in
// registers), else kMaxIter.
#define IC_LK_LAUNCH_KM(K, T, NJ, g, grid, threads, stream, ...)                            \
  do {                                                                                      \
    if ((g).iterations <= 4)                                                                \
      ::ic::lk::K<T, NJ, 4><<<(grid), (threads), 0, (stream)>>>(__VA_ARGS__);               \
    else                                                                                    \
      ::ic::lk::K<T, NJ, ::ic::lk::kMaxIter><<<(grid), (threads), 0, (stream)>>>(__VA_ARGS__); \
  } while (0)
#define IC_LK_LAUNCH(K, T, g, grid, threads, stream, ...)                                   \
  do {                                                                                      \
    switch ((g).J) {                                                                        \
      case 2: IC_LK_LAUNCH_KM(K, T, 2, g, grid, threads, stream, __VA_ARGS__); break;       \
      case 3: IC_LK_LAUNCH_KM(K, T, 3, g, grid, threads, stream, __VA_ARGS__); break;       \
      case 4: IC_LK_LAUNCH_KM(K, T, 4, g, grid, threads, stream, __VA_ARGS__); break;       \
      default: throw ::ic::ApiError(IC_ERR_INVALID_ARG, "lightcone snapshots must be 2 to 4"); \
    }                                                                                       \
  } while (0)

// Snapshot cotangents (in the snapshot's order) into the reverse sweep:
// dbar[t] += cd sd[a], pbar[t] += cp sp[a] with t = dest[a] (the slot in the
// next order), or t = a when dest is null; dbar may be null.  Targets are
// distinct, so no atomics.
template <typename T>
__global__ __launch_bounds__(256) void k_inject(const unsigned* __restrict__ dest,
                                                const T* __restrict__ sbar, T* __restrict__ dbar,
                                                T* __restrict__ pbar, T cd, T cp, long long P) {
  for (long long a = blockIdx.x * (long long)blockDim.x + threadIdx.x; a < P;
       a += (long long)gridDim.x * blockDim.x) {
    const long long t = dest ? static_cast<long long>(dest[a]) : a;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (dbar) dbar[q * P + t] += cd * sbar[q * P + a];
      pbar[q * P + t] += cp * sbar[(3 + q) * P + a];
    }
  }
}

}  // namespace lk
}  // namespace ic
