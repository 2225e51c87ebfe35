// Engine members for rank-order matching (paper section 2.3.2) and the
// projected L-BFGS iteration (section 2.3.1).  Included by engine_impl.h.
#pragma once

#include "rom.h"

namespace ic {

namespace ek {
// Count of entries of v below thr -> part[block] (FP64 counts).
static __global__ __launch_bounds__(fk::kRedThreads) void k_count_below(const uint32_t* __restrict__ v,
                                                                 uint32_t thr,
                                                                 double* __restrict__ part,
                                                                 long long n) {
  __shared__ double sh[fk::kRedThreads / 64];
  double c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if (v[i] < thr) c += 1.0;
  c = fk::block_sum(c, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

static __global__ void k_u64_to_u32(const uint64_t* __restrict__ a, uint32_t* __restrict__ b,
                             long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = static_cast<uint32_t>(a[i]);
}

static __global__ void k_fill_u32(uint32_t* __restrict__ a, uint32_t v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    a[i] = v;
}
}  // namespace ek

// Real space: the cells with R >= r_min, ranked by the white noise in
// descending order (ties by cell index), receive the sorted N(0,1) targets.
template <typename T>
long long Engine<T>::rom_real(T* s, uint64_t event) {
  const unsigned G = grid_for(P_, kThreads);
  const int vbits = 8 * sizeof(T);
  rk::k_real_keys<T><<<G, kThreads, 0, st_>>>(s, resp_, static_cast<T>(prob_.r_min), keys_,
                                              vals_, small_, P_);
  IC_LAUNCHED();
  radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, P_, vbits, st_);
  sk::k_gather_u32_key<<<G, kThreads, 0, st_>>>(small_, vals_, keys_, P_);
  IC_LAUNCHED();
  radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, P_, 4, st_);
  const unsigned g = grid_for(P_, fk::kRedThreads, kRedBlocks);
  ek::k_count_below<<<g, fk::kRedThreads, 0, st_>>>(small_, 1u, part_, P_);
  IC_LAUNCHED();
  double cnt = 0;
  reduce_parts(g, 1, &cnt);
  const long long n = (long long)cnt;
  dbg_n_[0] = n;
  if (n == 0) return 0;
  IC_HIP(hipMemcpyAsync(dbg_idx_[0], vals_, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st_));
  rk::k_gather<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(s, dbg_idx_[0], dbg_key_[0], n);
  IC_LAUNCHED();
  rk::k_real_targets<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(event, prob_.seed, tbuf_,
                                                                      keys_, vals_, n);
  IC_LAUNCHED();
  radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, n, vbits, st_);
  rk::k_scatter_sorted<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(s, dbg_idx_[0], tbuf_,
                                                                        vals_, n);
  IC_LAUNCHED();
  return n;
}

// Fourier space: z = rfft(s) / N^(3/2); independent modes with |k| >= k_min
// are matched per equal-width k bin.  Amplitude reading: ranked by |z| (ties
// by half-spectrum index), they get the sorted Rayleigh targets of their
// bin, phases kept.  Real/imaginary-part reading (reim): the 2n parts of a
// bin's n modes, ranked by value (ties by element index 2 f + c), get the
// sorted N(0, 1/2) targets of their bin.  Conjugate partners are mirrored
// before the inverse transform.  Returns the number of matched modes.
template <typename T>
long long Engine<T>::rom_fourier(T* s, uint64_t event, int32_t* bins_used, bool reim) {
  auto f = fa(0);
  cx<T>* Z = pool_;
  fft_r2c_z<T>(f, s, T(1), nullptr, T(0), Z);
  fft_y<T>(f, Z, true);
  fft_x<T>(f, Z, Z, true, T(1));
  const double n3h = std::pow((double)np_, 1.5);
  const int nbins = prob_.rom_nbins;
  if (nbins < 1 || nbins > 127) throw ApiError(IC_ERR_INVALID_ARG, "rom_nbins must be in [1, 127]");
  const double kf = 2.0 * 3.14159265358979323846 / prob_.box;
  const double kmax = std::sqrt(3.0) * 3.14159265358979323846 * np_ / prob_.box;
  const double dk = (kmax - prob_.rom_kmin) / nbins;
  const long long E = reim ? 2 * Hq_ : Hq_;  // ranked elements
  const unsigned G = grid_for(Hq_, kThreads);
  const unsigned GE = grid_for(E, kThreads);
  const int vbits = 8 * sizeof(T);
  if (reim)
    rk::k_part_keys<T><<<G, kThreads, 0, st_>>>(Z, np_, kpp_, static_cast<T>(1.0 / n3h), kf,
                                                prob_.rom_kmin, dk, nbins, vbuf_, keys_, vals_,
                                                small_, Hq_);
  else
    rk::k_mode_keys<T><<<G, kThreads, 0, st_>>>(Z, np_, kpp_, static_cast<T>(1.0 / n3h), kf,
                                                prob_.rom_kmin, dk, nbins, vbuf_, keys_, vals_,
                                                small_, Hq_);
  IC_LAUNCHED();
  radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, E, vbits, st_);
  sk::k_gather_u32_key<<<GE, kThreads, 0, st_>>>(small_, vals_, keys_, E);
  IC_LAUNCHED();
  radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, E, 8, st_);
  ek::k_fill_u32<<<1, 256, 0, st_>>>(binc_, 0u, 256);
  IC_LAUNCHED();
  rk::k_bin_ends<<<GE, kThreads, 0, st_>>>(keys_, binc_, E);
  IC_LAUNCHED();
  std::vector<uint32_t>& counts = bin_count_;
  IC_HIP(hipMemcpyAsync(counts.data(), binc_, 256 * sizeof(uint32_t), hipMemcpyDeviceToHost, st_));
  IC_HIP(hipStreamSynchronize(st_));
  // run ends -> counts (bins are sorted ascending; absent bins read 0)
  for (uint32_t b = 0, prev = 0; b < 255; ++b) {
    if (counts[b] == 0) continue;
    const uint32_t e = counts[b];
    counts[b] = e - prev;
    prev = e;
  }
  std::vector<uint32_t>& start = bin_start_;
  std::fill(start.begin(), start.end(), 0u);
  long long n = 0;
  int used = 0;
  for (int b = 0; b < nbins; ++b) {
    start[b] = static_cast<uint32_t>(n);
    n += counts[b];
    used += counts[b] > 0;
  }
  if (bins_used) *bins_used = used;
  dbg_n_[1] = n;
  if (n > 0) {
    IC_HIP(hipMemcpyAsync(binc_ + 128, start.data(), 128 * sizeof(uint32_t),
                          hipMemcpyHostToDevice, st_));
    IC_HIP(hipMemcpyAsync(dbg_idx_[1], vals_, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st_));
    const unsigned Gn = grid_for(n, kThreads);
    ek::k_u64_to_u32<<<Gn, kThreads, 0, st_>>>(keys_, dbg_bin_, n);
    IC_LAUNCHED();
    rk::k_gather<T><<<Gn, kThreads, 0, st_>>>(vbuf_, dbg_idx_[1], dbg_key_[1], n);
    IC_LAUNCHED();
    // Rayleigh draws (stream 3) for amplitudes; N(0, 1/2) draws (stream 5)
    // for the parts
    rk::k_fourier_targets<T><<<Gn, kThreads, 0, st_>>>(
        keys_, binc_ + 128, reim ? 0 : 1, reim ? 5 : 3, reim ? std::sqrt(0.5) : 1.0, event,
        prob_.seed, tbuf_, keys_, vals_, small_, n);
    IC_LAUNCHED();
    radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, n, vbits, st_);
    sk::k_gather_u32_key<<<Gn, kThreads, 0, st_>>>(small_, vals_, keys_, n);
    IC_LAUNCHED();
    radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, n, 8, st_);
    if (reim) {
      rk::k_part_scatter<T><<<Gn, kThreads, 0, st_>>>(Z, np_, kpp_, dbg_idx_[1], tbuf_, vals_,
                                                      static_cast<T>(n3h), n);
      IC_LAUNCHED();
      rk::k_part_mirror<T><<<Gn, kThreads, 0, st_>>>(Z, np_, kpp_, dbg_idx_[1], n);
      IC_LAUNCHED();
    } else {
      rk::k_fourier_scatter<T><<<Gn, kThreads, 0, st_>>>(Z, np_, kpp_, dbg_idx_[1], tbuf_,
                                                         vals_, static_cast<T>(n3h), n);
      IC_LAUNCHED();
    }
  }
  fft_x<T>(f, Z, Z, false, static_cast<T>(1.0 / (double)P_));
  fft_y<T>(f, Z, false);
  fft_c2r_z<T>(f, Z, s, T(1), nullptr, T(0));
  return reim ? n / 2 : n;
}

template <typename T>
void Engine<T>::lbfgs_step(void* sv, void* gv, double* loss, int64_t it, ic_lbfgs_info* info) {
  if (!sv || !gv || !loss) throw ApiError(IC_ERR_INVALID_ARG, "null argument");
  if (!counts_) throw ApiError(IC_ERR_STATE, "no observation set");
  T* s = static_cast<T*>(sv);
  T* g = static_cast<T*>(gv);
  require_finite(s, "s");
  const double L = *loss;
  if (!std::isfinite(L)) throw ApiError(IC_ERR_NONFINITE, "loss is not finite");
  const int m = prob_.lbfgs_m;
  ic_lbfgs_info inf{};
  // Two-loop recursion: dir = -H g with H0 = gamma I; gamma = S.Y / Y.Y of
  // the newest pair, or 1 / |g| with an empty history (a unit-length first step).
  const double gnorm = std::sqrt(dot(g, g, P_));
  if (!std::isfinite(gnorm)) throw ApiError(IC_ERR_NONFINITE, "gradient is not finite");
  if (!(gnorm > 0)) throw ApiError(IC_ERR_LINESEARCH, "zero gradient: no descent direction");
  const int h = static_cast<int>(hist_.size());
  const double gamma = h ? hist_sy_[hist_.back()] / hist_yy_[hist_.back()] : 1.0 / gnorm;
  double gp;
  if (h == 0) {
    scale(g, -gamma, dir_, P_);  // -g / |g|
    gp = dot(g, dir_, P_);
  } else {
    // Fused recursion: every step updates the direction and reduces the dot
    // product the next step needs into lbs_ on the device, so the host waits
    // once, for g.p.  A[i] = S_i . q (lbs_[i]), B[i] = Y_i . r (lbs_[64 + i]),
    // alpha_i = rho_i A[i], beta_i = rho_i B[i] (times gamma for i = 0, whose
    // dot is taken before the scaling r = gamma q).
    const unsigned G = grid_for(P_, fk::kRedThreads, kRedBlocks);
    auto S = [&](int i) { return hist_S_ + hist_[i] * P_; };
    auto Y = [&](int i) { return hist_Y_ + hist_[i] * P_; };
    auto rho = [&](int i) { return hist_rho_[hist_[i]]; };
    auto reduce_to = [&](double* dst) {
      fk::k_reduce_parts<<<1, fk::kRedThreads, 0, st_>>>(part_, G, 1, dst);
      IC_LAUNCHED();
    };
    fk::k_dot<T><<<G, fk::kRedThreads, 0, st_>>>(S(h - 1), g, part_, P_);
    IC_LAUNCHED();
    reduce_to(lbs_ + (h - 1));
    for (int i = h - 1; i >= 0; --i) {  // q -= alpha_i Y_i
      const T* in = i == h - 1 ? g : dir_;
      const T* V = i > 0 ? S(i - 1) : Y(0);
      fk::k_lbfgs_update<T><<<G, fk::kRedThreads, 0, st_>>>(
          in, T(1), Y(i), lbs_, i, -1, -rho(i), 0.0, dir_, V, part_, P_);
      IC_LAUNCHED();
      reduce_to(i > 0 ? lbs_ + (i - 1) : lbs_ + 64);
    }
    for (int i = 0; i < h; ++i) {  // r += (alpha_i - beta_i) S_i; p = -r at the end
      const bool last = i == h - 1;
      const T sgn = last ? T(-1) : T(1);
      const T s_in = sgn * static_cast<T>(i == 0 ? gamma : 1.0);
      fk::k_lbfgs_update<T><<<G, fk::kRedThreads, 0, st_>>>(
          dir_, s_in, S(i), lbs_, i, 64 + i, static_cast<double>(sgn) * rho(i),
          i == 0 ? gamma : 1.0, dir_, last ? g : Y(i + 1), part_, P_);
      IC_LAUNCHED();
      if (!last) reduce_to(lbs_ + 64 + i + 1);
    }
    double r = 0;
    reduce_parts(G, 1, &r);
    gp = r;
  }
  if (!(gp < 0)) {
    lbfgs_reset();
    scale(g, -1.0 / gnorm, dir_, P_);
    gp = dot(g, dir_, P_);
    inf.restarted = 1;
  }
  // Backtracking along the projection arc: accept s' = P(s + eps p) when
  // g.(s' - s) < 0, L(s') < L and L(s') <= L + c1 g.(s' - s).  A quasi-Newton direction
  // whose search fails is replaced once by steepest descent (history reset),
  // with trial numbers continuing after max_trials.  Without projected steps
  // (project_steps = 0) s' = s + eps p: plain backtracking L-BFGS.
  double eps = 0;
  bool accepted = false;
  ic_loss_terms t{};
  int used = 0;
  for (int attempt = 0; attempt < 2 && !accepted; ++attempt) {
    if (attempt == 1) {
      if (hist_.empty()) break;
      lbfgs_reset();
      scale(g, -1.0 / gnorm, dir_, P_);
      gp = dot(g, dir_, P_);
      inf.restarted = 1;
    }
    eps = prob_.eps_max;
    for (int k = 0; k < prob_.max_trials; ++k) {
      const int trial = attempt * prob_.max_trials + k;
      axpy(s, dir_, eps, strial_, P_);
      inf.resets = prob_.project_steps ? project(strial_, strial_, (uint64_t)trial, (uint64_t)it)
                                       : 0;
      eval(strial_, gtrial_, &t);
      inf.evaluations++;
      used = k + 1;
      const double dec = dot_diff(g, strial_, s);
      if (dec < 0 && t.loss < L && t.loss <= L + prob_.armijo_c1 * dec) {
        accepted = true;
        break;
      }
      eps *= 0.5;
    }
  }
  inf.trials = used;
  inf.gp = gp;
  if (!accepted) {
    if (info) *info = inf;
    throw ApiError(IC_ERR_LINESEARCH, "line search found no acceptable step");
  }
  inf.eps = eps;
  const int sl = free_slots_.back();
  T* Sv = hist_S_ + sl * P_;
  T* Yv = hist_Y_ + sl * P_;
  fk::k_sub<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(strial_, s, Sv, P_);
  IC_LAUNCHED();
  fk::k_sub<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(gtrial_, g, Yv, P_);
  IC_LAUNCHED();
  const double sy = dot(Sv, Yv, P_), ss = dot(Sv, Sv, P_), yy = dot(Yv, Yv, P_);
  if (sy > 1e-10 * std::sqrt(ss * yy)) {
    free_slots_.pop_back();
    hist_.push_back(sl);
    hist_rho_[sl] = 1.0 / sy;
    hist_sy_[sl] = sy;
    hist_yy_[sl] = yy;
    if ((int)hist_.size() > m) {
      free_slots_.push_back(hist_.front());
      hist_.pop_front();
    }
    inf.stored = 1;
  }
  inf.history = static_cast<int32_t>(hist_.size());
  copy(strial_, s, P_);
  copy(gtrial_, g, P_);
  *loss = t.loss;
  IC_HIP(hipStreamSynchronize(st_));
  if (info) *info = inf;
}

}  // namespace ic
