// Hot-path engine for one element type: forward model, hand-written adjoint,
// projection, rank-order matching and projected L-BFGS on the caller's
// workspace.  Included once per precision.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <string>
#include <vector>

#include "cosmo.h"
#include "engine.h"
#include "fft.h"
#include "fields.h"
#include "blocks.h"
#include "lightcone.h"
#include "particles.h"
#include "sort.h"
#include "timer.h"

namespace ic {

// Sequential 256-byte-aligned carving of the caller's workspace (base == nullptr
// only measures).
class Carver {
 public:
  explicit Carver(char* base) : base_(base) {}
  template <typename X>
  X* take(size_t count) {
    off_ = (off_ + 255) & ~size_t(255);
    X* p = base_ ? reinterpret_cast<X*>(base_ + off_) : nullptr;
    off_ += count * sizeof(X);
    return p;
  }
  size_t used() const { return (off_ + 255) & ~size_t(255); }

 private:
  char* base_;
  size_t off_ = 0;
};

inline int ilog2(long long v) {
  int l = 0;
  while ((1ll << l) < v) ++l;
  return l;
}

template <typename T>
class Engine final : public EngineBase {
 public:
  static constexpr unsigned kThreads = 256;
  static constexpr unsigned kRedBlocks = 4096;

  Engine(const ic_problem& p, char* ws, size_t ws_bytes, hipStream_t stream)
      : prob_(p), st_(stream) {
    np_ = p.n_part;
    nm_ = p.n_mesh;
    S_ = p.n_steps;
    lp_ = ilog2(np_);
    lm_ = ilog2(nm_);
    ratio_ = nm_ / np_;
    P_ = (long long)np_ * np_ * np_;
    M_ = (long long)nm_ * nm_ * nm_;
    kpp_ = spectrum_pitch<T>(np_);
    kpm_ = spectrum_pitch<T>(nm_);
    Hp_ = (long long)np_ * np_ * kpp_;
    Hm_ = (long long)nm_ * nm_ * kpm_;
    Hq_ = (long long)np_ * np_ * (np_ / 2 + 1);
    tape_forces_ = p.tape_forces != 0;
    // Checkpoint spacing; a spacing beyond the last step keeps state 0 only.
    K_ = p.ckpt_every > 0 ? std::min(p.ckpt_every, S_ + 1) : 0;
    Lm_ = bk::layout_for(lm_);
    Ld_ = bk::layout_for(lp_);
    nbm_ = bk::block_count(Lm_);
    nbd_ = bk::block_count(Ld_);
    mim_ = bk::max_items(Lm_, P_);
    mid_ = bk::max_items(Ld_, P_);
    const int m = std::max(1, p.lbfgs_m);
    wtab_len_ = 3 * (np_ / 2) * (np_ / 2) + 1;
    // sort length of rank-order matching: the field, or the 2 n^2 (n/2+1)
    // real and imaginary parts of the half spectrum (IC_ROM_FOURIER_REIM)
    rom_len_ = std::max(P_, 2 * Hq_);
    sort_blocks_ = (rom_len_ + sk::kTile - 1) / sk::kTile;

    Carver c(ws);
    twp_ = c.take<cx<T>>(np_);
    twm_ = c.take<cx<T>>(nm_);
    wtab_ = c.take<T>(wtab_len_);
    pool_len_ = std::max(10 * Hp_, 4 * Hm_);
    pool_ = c.take<cx<T>>(pool_len_);
    phi_ = c.take<T>(6 * P_);
    mu_ = c.take<T>(P_);
    // Particle states: every step's positions (K_ = 0), or positions and
    // momenta at the checkpoints 0, K, 2K, ... plus K - 1 slots for the
    // states between two checkpoints.  Force meshes: one per kept state.
    const long long nck = K_ ? S_ / K_ + 1 : 0;
    dtape_ = c.take<T>((K_ ? nck + K_ - 1 : S_ + 1) * 3 * P_);
    ckp_ = K_ ? c.take<T>(nck * 3 * P_) : nullptr;
    gtape_ = c.take<T>((tape_forces_ ? (K_ ? K_ : S_ + 1) : 1) * 3 * M_);
    p_ = c.take<T>(3 * P_);
    rhom_ = c.take<T>(M_);
    rhod_ = c.take<T>(P_);
    seed_ = c.take<T>(P_);
    dbar_ = c.take<T>(3 * P_);
    pbar_ = c.take<T>(3 * P_);
    gbar_ = c.take<T>(3 * M_);
    rhobar_ = c.take<T>(M_);
    part_ = c.take<double>(3 * kRedBlocks);
    scal_ = c.take<double>(64);
    lbs_ = c.take<double>(2 * 64);  // two-loop dot products left on the device
    hist_S_ = c.take<T>((size_t)(m + 1) * P_);
    hist_Y_ = c.take<T>((size_t)(m + 1) * P_);
    dir_ = c.take<T>(P_);
    strial_ = c.take<T>(P_);
    gtrial_ = c.take<T>(P_);
    keys_ = c.take<uint64_t>(rom_len_);
    keys2_ = c.take<uint64_t>(rom_len_);
    vals_ = c.take<uint32_t>(rom_len_);
    vals2_ = c.take<uint32_t>(rom_len_);
    small_ = c.take<uint32_t>(rom_len_);
    shist_ = c.take<uint32_t>(sk::kDigits * sort_blocks_);
    vbuf_ = c.take<T>(rom_len_);
    tbuf_ = c.take<T>(rom_len_);
    binc_ = c.take<uint32_t>(256);
    // Block orders of the particles: one per mesh state d_0..d_S, one on the
    // data grid; ids and dest per order (see blocks.h).
    idtape_ = c.take<uint32_t>((size_t)(S_ + 1) * P_);
    desttape_ = c.take<uint32_t>((size_t)(S_ + 2) * P_);
    ostart_ = c.take<uint32_t>((size_t)(S_ + 1) * (nbm_ + 1));
    oistart_ = c.take<uint32_t>((size_t)(S_ + 1) * (nbm_ + 1));
    oitems_ = c.take<uint2>((size_t)(S_ + 1) * mim_);
    dstart_ = c.take<uint32_t>(nbd_ + 1);
    distart_ = c.take<uint32_t>(nbd_ + 1);
    ditems_ = c.take<uint2>(mid_);
    dids_ = c.take<uint32_t>(P_);
    bcount_ = c.take<uint32_t>(std::max(nbm_, nbd_));
    bkey_ = c.take<uint32_t>(P_);
    brank_ = c.take<uint32_t>(P_);
    pinv_ = c.take<uint32_t>(P_);
    bsums_ = c.take<uint2>(1024);
    // halos of the paints (blocks.h): the x/y staging, one slot of
    // nf x kHaloXY values per work item (three fields on the mesh orders, one
    // on the data order); the z halos, one value per eight cells of each
    // painted field (three mesh fields; the data grid's apart, since the
    // loss reads it after the adjoint's paints began)
    hstage_ = c.take<T>((size_t)std::max<long long>(3ll * mim_, mid_) * bk::kHaloXY);
    det_ = p.deterministic != 0;
    if (det_) {
      // deterministic mode: the paints' integer fields (three mesh fields, or
      // the data grid), their z halo and x/y halo staging, and the device
      // maximum the cotangent paint's scale is chosen for
      det64_ = c.take<unsigned long long>(3 * std::max(M_, P_));
      detzh_ = c.take<unsigned long long>(3 * std::max(M_, P_) / kZHalo);
      detstage_ =
          c.take<unsigned long long>((size_t)std::max<long long>(3ll * mim_, mid_) * bk::kHaloXY);
      detvmax_ = c.take<double>(8);
    }
    zh_ = c.take<T>(3 * M_ / kZHalo);
    zhd_ = c.take<T>(P_ / kZHalo);
    tmpd_ = c.take<T>(3 * P_);
    tmpp_ = c.take<T>(3 * P_);
    dsd_ = c.take<T>(3 * P_);
    psd_ = c.take<T>(3 * P_);
    dbar2_ = c.take<T>(3 * P_);
    pbar2_ = c.take<T>(3 * P_);
    dbg_idx_[0] = c.take<uint32_t>(P_);
    dbg_key_[0] = c.take<T>(P_);
    dbg_idx_[1] = c.take<uint32_t>(2 * Hq_);
    dbg_key_[1] = c.take<T>(2 * Hq_);
    dbg_bin_ = c.take<uint32_t>(2 * Hq_);
    // Lightcone: the snapshots before the last (each in its step's order, 6
    // fields), their snapshot slots in the final order,
    // their cotangents, and the inverse comoving-distance table.
    lc_on_ = p.lc_n >= 2;
    if (lc_on_) {
      for (int j = 0; j + 1 < p.lc_n; ++j) lc_steps_.push_back(snapshot_step(p, p.lc_a[j]));
      snap_ = c.take<T>(lc_steps_.size() * 6 * P_);
      snapbar_ = c.take<T>(lc_steps_.size() * 6 * P_);
      snapinv_ = c.take<uint32_t>(lc_steps_.size() * P_);
      lct_ = c.take<double>(2 * kLcNodes);
    }
    need_ = c.used();
    if (!ws) return;
    if (ws_bytes < need_) throw ApiError(IC_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
      throw ApiError(IC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (det_ && !(det64_ && detzh_ && detstage_ && detvmax_))
      throw ApiError(IC_ERR_STATE, "deterministic-mode buffers missing from the workspace");
    timer_.set_stream(st_);
    for (int i = 0; i <= m; ++i) free_slots_.push_back(i);

    CosmoParams cp{p.omega_m, p.h, p.n_s, p.sigma8, p.a_init, p.a_final, p.n_steps};
    co_ = compute_coeffs(cp);
    std::vector<double> w = whitening_table(cp, co_.pk_amplitude, p.box, np_);
    std::vector<T> wt(w.begin(), w.end());
    std::vector<cx<T>> tp = twiddles(np_), tm = twiddles(nm_);
    IC_HIP(hipMemcpyAsync(wtab_, wt.data(), wt.size() * sizeof(T), hipMemcpyHostToDevice, st_));
    IC_HIP(hipMemcpyAsync(twp_, tp.data(), tp.size() * sizeof(cx<T>), hipMemcpyHostToDevice, st_));
    IC_HIP(hipMemcpyAsync(twm_, tm.data(), tm.size() * sizeof(cx<T>), hipMemcpyHostToDevice, st_));
    if (lc_on_) {
      const double a_lo = co_.a[lc_steps_[0]];  // the first snapshot's step
      const LightconeTable t = lightcone_table(p.omega_m, a_lo, p.a_final, kLcNodes);
      IC_HIP(hipMemcpyAsync(lct_, t.a.data(), kLcNodes * sizeof(double), hipMemcpyHostToDevice,
                            st_));
      IC_HIP(hipMemcpyAsync(lct_ + kLcNodes, t.slope.data(), kLcNodes * sizeof(double),
                            hipMemcpyHostToDevice, st_));
      lk::LcGeo& g = lcgeo_;
      for (int j = 0; j < lk::kMaxSnap; ++j) g.a_snap[j] = j < p.lc_n ? p.lc_a[j] : 0.0;
      g.a_snap[p.lc_n - 1] = p.a_final;
      for (int j = 0; j + 1 < p.lc_n; ++j) g.a_snap[j] = co_.a[lc_steps_[j]];
      g.J = p.lc_n;
      g.iterations = p.lc_iterations;
      g.om = p.omega_m;
      g.c_final = co_.rsd_factor;
      g.tab = lk::LcTable{lct_, lct_ + kLcNodes, t.chi_min, t.chi_max, t.h, 1.0 / t.h,
                          kLcNodes, a_lo, p.a_final};
    }
    IC_HIP(hipStreamSynchronize(st_));
  }

  size_t needed() const { return need_; }

  // ------------------------------------------------------------ interface
  void set_stream(hipStream_t s) override {
    st_ = s;
    timer_.set_stream(s);
  }

  hipStream_t stream() const override { return st_; }
  const ic_problem& problem() const override { return prob_; }

  void set_observation(const int32_t* counts, const void* response) override {
    if (!counts || !response) throw ApiError(IC_ERR_INVALID_ARG, "null observation buffer");
    counts_ = counts;
    resp_ = static_cast<const T*>(response);
  }

  // Non-finite white noise is refused before any particle is moved.
  void require_finite(const void* x, const char* what) {
    if (count_nonfinite(static_cast<const T*>(x), P_) > 0)
      throw ApiError(IC_ERR_NONFINITE, std::string(what) + " is not finite");
  }

  void forward(const void* s, void* delta, void* lambda, double* loss) override {
    if (!s) throw ApiError(IC_ERR_INVALID_ARG, "s is null");
    if (loss && !counts_) throw ApiError(IC_ERR_STATE, "no observation set");
    if (lambda && !resp_) throw ApiError(IC_ERR_STATE, "no observation set");
    require_finite(s, "s");
    run_forward(static_cast<const T*>(s));
    if (delta || lambda || loss) {
      ic_loss_terms t{};
      observe(static_cast<const T*>(s), static_cast<T*>(delta), static_cast<T*>(lambda),
              loss ? &t : nullptr, loss != nullptr);
      if (loss) *loss = t.loss;
    }
  }

  void loss_and_grad(const void* s, void* grad, ic_loss_terms* terms) override {
    if (!s || !grad) throw ApiError(IC_ERR_INVALID_ARG, "null buffer");
    if (!counts_) throw ApiError(IC_ERR_STATE, "no observation set");
    require_finite(s, "s");
    ic_loss_terms t{};
    eval(static_cast<const T*>(s), static_cast<T*>(grad), &t);
    if (terms) *terms = t;
    if (!std::isfinite(t.loss)) throw ApiError(IC_ERR_NONFINITE, "loss is not finite");
    if (count_nonfinite(static_cast<const T*>(grad), P_) > 0)
      throw ApiError(IC_ERR_NONFINITE, "gradient is not finite");
  }

  void vjp(const void* s, const void* delta_bar, void* s_bar) override {
    if (!s || !delta_bar || !s_bar) throw ApiError(IC_ERR_INVALID_ARG, "null buffer");
    require_finite(s, "s");
    run_forward(static_cast<const T*>(s));
    copy(static_cast<const T*>(delta_bar), seed_, P_);
    adjoint(static_cast<T*>(s_bar), nullptr, T(0));
  }

  void project_rankmatch(void* sv, uint32_t flags, uint64_t event, int32_t trial,
                         ic_rom_info* info) override {
    if (!sv) throw ApiError(IC_ERR_INVALID_ARG, "s is null");
    T* s = static_cast<T*>(sv);
    ic_rom_info inf{};
    if (flags & (IC_ROM_REAL | IC_ROM_FOURIER | IC_ROM_FOURIER_REIM)) {
      if (count_nonfinite(s, P_) > 0) throw ApiError(IC_ERR_NONFINITE, "non-finite input to matching");
    }
    if (flags & IC_ROM_REAL) {
      if (!resp_) throw ApiError(IC_ERR_STATE, "real-space matching needs the response field");
      inf.n_real = rom_real(s, event);
    }
    if ((flags & IC_ROM_FOURIER) && (flags & IC_ROM_FOURIER_REIM))
      throw ApiError(IC_ERR_INVALID_ARG,
                     "IC_ROM_FOURIER and IC_ROM_FOURIER_REIM are alternative readings");
    if (flags & (IC_ROM_FOURIER | IC_ROM_FOURIER_REIM))
      inf.n_fourier = rom_fourier(s, event, &inf.bins_used, (flags & IC_ROM_FOURIER_REIM) != 0);
    if (flags & IC_PROJECT) inf.resets = project(s, s, (uint64_t)trial, event);
    if (info) *info = inf;
  }

  void lbfgs_step(void* sv, void* gv, double* loss, int64_t it, ic_lbfgs_info* info) override;

  void lbfgs_reset() override {
    free_slots_.insert(free_slots_.end(), hist_.begin(), hist_.end());
    hist_.clear();
  }

  // Fresh N(0,1) noise on this grid (Philox stream 4, counter (j, 0, 4, event),
  // j the lattice index) whose modes inside the coarse band are replaced by
  // the coarse field's, scaled.  The coarse forward transform runs on the
  // low engine, on this engine's stream, into spare space of this engine's
  // spectrum pool.
  void upsample_from(EngineBase& low, const void* s_low, void* s_high,
                     uint64_t event) override {
    const ic_problem& lp = low.problem();
    const int nl = lp.n_part;
    if (nl * 2 != np_ || lp.box != prob_.box)
      throw ApiError(IC_ERR_INVALID_ARG,
                     "the coarse context needs half the particle grid side and the same box");
    if (!s_low || !s_high) throw ApiError(IC_ERR_INVALID_ARG, "null field");
    cx<T>* zl = pool_ + Hp_;  // dense coarse half spectrum (nl^2 (nl/2+1) < Hp_ entries)
    const hipStream_t ls = low.stream();
    low.set_stream(st_);
    try {
      low.op_rfft(0, s_low, zl);
    } catch (...) {
      low.set_stream(ls);
      throw;
    }
    low.set_stream(ls);
    T* out = static_cast<T*>(s_high);
    fk::k_philox<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(0, 0, 4, event, prob_.seed,
                                                                  out, P_);
    IC_LAUNCHED();
    auto f = fa(0);
    fft_r2c_z<T>(f, out, T(1), nullptr, T(0), pool_);
    fft_y<T>(f, pool_, true);
    fft_x<T>(f, pool_, pool_, true, T(1));
    const long long modes = (long long)nl * nl * (nl / 2);
    fk::k_embed_coarse<T><<<grid_for(modes, kThreads), kThreads, 0, st_>>>(
        zl, nl, pool_, np_, kpp_, static_cast<T>(std::pow((double)np_ / nl, 1.5)));
    IC_LAUNCHED();
    fft_x<T>(f, pool_, pool_, false, T(1.0 / (double)P_));
    fft_y<T>(f, pool_, false);
    fft_c2r_z<T>(f, pool_, out, T(1), nullptr, T(0));
  }

  // Spectra cross the ABI in the contiguous n x n x (n/2+1) layout.
  void op_rfft(int grid, const void* x, void* xk) override {
    auto f = fa(grid);
    {
      auto sc = timer_.scope("fft_r2c_z", 0);
      fft_r2c_z<T>(f, static_cast<const T*>(x), T(1), nullptr, T(0), pool_);
    }
    fft_y<T>(f, pool_, true);
    fft_x<T>(f, pool_, pool_, true, T(1));
    spectrum_pack<T>(f, pool_, static_cast<cx<T>*>(xk));
  }

  void op_irfft(int grid, const void* xk, void* x) override {
    auto f = fa(grid);
    const long long n3 = grid ? M_ : P_;
    spectrum_unpack<T>(f, static_cast<const cx<T>*>(xk), pool_);
    fft_x<T>(f, pool_, pool_, false, T(1.0 / (double)n3));
    fft_y<T>(f, pool_, false);
    fft_c2r_z<T>(f, pool_, static_cast<T*>(x), T(1), nullptr, T(0));
  }

  void op_multiplier(int kinds, int a, int b, const void* x, void* y) override {
    if (a < 0 || a > 2 || b < 0 || b > 2) throw ApiError(IC_ERR_INVALID_ARG, "axis out of range");
    MulSpec sp;
    sp.kinds = kinds;
    sp.ga = a;
    sp.ha = a;
    sp.hb = b;
    sp.scale = 1.0 / (double)P_;
    T* outs[1] = {static_cast<T*>(y)};
    chain_scatter(0, static_cast<const T*>(x), T(1), nullptr, T(0), outs, &sp, 1);
  }

  void op_paint(int grid, const void* disp, void* rho) override {
    paint_lattice(static_cast<const T*>(disp), grid, static_cast<T*>(rho));
  }

  // The readout runs in the hot path's step kernel on the block order the
  // paint sorted the particles into: a kick of one from zero momentum with
  // no drift leaves the force itself as the new momentum, which goes back
  // to the lattice order.
  void op_force(const void* disp, void* force) override {
    const T* d = static_cast<const T*>(disp);
    paint_lattice(d, 1, rhom_, false);  // positions of order 0 in tmpd_, ids in dids_
    force_from_density(gtape_);         // adds the z halo left in zh_
    fill(tmpp_, T(0), 3 * P_);
    bk::k_step_b<T><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
        tmpd_, tmpp_, nullptr, gtape_, M_, T(1), T(0), P_, lp_, gmesh(), Lm_,
        items(mesh_order(0), dids_), dbar2_, pbar2_, nullptr, nullptr, nullptr);
    IC_LAUNCHED();
    T* F = static_cast<T*>(force);
    bk::k_to_lattice<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
        dids_, bk::Ptrs<T>{{pbar2_, pbar2_ + P_, pbar2_ + 2 * P_}},
        bk::MPtrs<T>{{F, F + P_, F + 2 * P_}}, 3, P_);
    IC_LAUNCHED();
  }

  void op_lpt(const void* s, void* d0, void* p0) override {
    lpt(static_cast<const T*>(s), static_cast<T*>(d0), static_cast<T*>(p0));
  }

  // Final state in lattice order.
  void op_evolve(const void* s, void* d, void* p) override {
    run_forward(static_cast<const T*>(s));
    T* dd = static_cast<T*>(d);
    T* pp = static_cast<T*>(p);
    bk::k_to_lattice<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
        ids(S_), state_ptrs(dslot(S_), pslot(S_)), state_mptrs(dd, pp), 6, P_);
    IC_LAUNCHED();
  }

  void op_sort_desc(const void* values, int64_t n, int32_t* order) override {
    if (n < 0 || n > P_) throw ApiError(IC_ERR_INVALID_ARG, "sort length out of range");
    if (n == 0) return;
    if (count_nonfinite(static_cast<const T*>(values), n) > 0)
      throw ApiError(IC_ERR_NONFINITE, "NaN in sort input");
    sk::k_desc_keys<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(
        static_cast<const T*>(values), keys_, vals_, n);
    IC_LAUNCHED();
    radix_sort_pairs(keys_, vals_, keys2_, vals2_, shist_, n, 8 * sizeof(T), st_);
    IC_HIP(hipMemcpyAsync(order, vals_, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st_));
  }

  void op_philox(int kind, uint64_t sub, uint64_t stream, uint64_t event, int64_t n,
                 void* out) override {
    if (n < 0) throw ApiError(IC_ERR_INVALID_ARG, "negative count");
    if (n == 0) return;
    fk::k_philox<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(
        kind, sub, stream, event, prob_.seed, static_cast<T*>(out), n);
    IC_LAUNCHED();
  }

  void debug_rom_order(int space, int32_t* idx, void* keys, int32_t* bins, int64_t cap,
                       int64_t* n) override {
    if (space < 0 || space > 1) throw ApiError(IC_ERR_INVALID_ARG, "space must be 0 or 1");
    const long long cnt = dbg_n_[space];
    if (cnt < 0) throw ApiError(IC_ERR_STATE, "no rank-order matching recorded");
    if (n) *n = cnt;
    if (cap < cnt) return;
    if (idx)
      IC_HIP(hipMemcpyAsync(idx, dbg_idx_[space], cnt * sizeof(uint32_t), hipMemcpyDeviceToHost, st_));
    if (keys)
      IC_HIP(hipMemcpyAsync(keys, dbg_key_[space], cnt * sizeof(T), hipMemcpyDeviceToHost, st_));
    if (bins && space == 1)
      IC_HIP(hipMemcpyAsync(bins, dbg_bin_, cnt * sizeof(uint32_t), hipMemcpyDeviceToHost, st_));
    IC_HIP(hipStreamSynchronize(st_));
  }

  void timing(bool enable) override { timer_.enable(enable); }
  void timing_only(const char* kernel) override {
    if (!kernel || !*kernel) throw ApiError(IC_ERR_INVALID_ARG, "kernel name required");
    timer_.enable(true, kernel);
  }
  std::string timing_report() override { return timer_.report(); }

 private:
  // ------------------------------------------------------------- helpers
  static std::vector<cx<T>> twiddles(int n) {
    std::vector<cx<T>> t(n);
    for (int m = 0; m < n; ++m) {
      // exp(-2 pi i m / n), evaluated in FP64 and rounded once to T.
      const double ang = 2.0 * 3.14159265358979323846 * (double)m / (double)n;
      t[m] = mkc<T>(static_cast<T>(std::cos(ang)), static_cast<T>(-std::sin(ang)));
    }
    return t;
  }

  // Algorithmic bytes of one half spectrum of side n (the row padding of the
  // stored layout is not counted).
  double half_spectrum_bytes(int n) const {
    return (double)n * n * (n / 2 + 1) * 2 * sizeT();
  }

  FftArgs<T> fa(int grid) const {
    FftArgs<T> f;
    f.n = grid ? nm_ : np_;
    f.kp = grid ? kpm_ : kpp_;
    f.tw = grid ? twm_ : twp_;
    f.wtab = wtab_;
    f.box = prob_.box;
    f.stream = st_;
    return f;
  }

  pk::Grid<T> gmesh() const {
    return {lm_, ratio_, static_cast<T>((double)nm_ / prob_.box), static_cast<T>(prob_.box / nm_)};
  }
  pk::Grid<T> gdata() const {
    return {lp_, 1, static_cast<T>((double)np_ / prob_.box), static_cast<T>(prob_.box / np_)};
  }

  pk::Rsd<T> rsd() const {
    pk::Rsd<T> r;
    r.mode = prob_.rsd_mode;
    r.n = np_;
    r.c = static_cast<T>(co_.rsd_factor);
    r.box = static_cast<T>(prob_.box);
    r.dq = static_cast<T>(prob_.box / np_);
    for (int a = 0; a < 3; ++a) r.obs[a] = static_cast<T>(prob_.observer[a]);
    return r;
  }

  // Slots of state n: positions d_n, the momentum the step from n starts
  // with, and the force meshes at d_n.  With checkpoints, states K j sit in
  // their own slots (d then the checkpoint area's first S/K + 1 slots) and
  // the others share K - 1 segment slots.
  T* dslot(int n) const {
    if (!K_) return dtape_ + (long long)n * 3 * P_;
    const long long nck = S_ / K_ + 1;
    const long long j = n % K_ == 0 ? n / K_ : nck + n % K_ - 1;
    return dtape_ + j * 3 * P_;
  }
  T* pslot(int n) const {
    return K_ && n % K_ == 0 ? ckp_ + (long long)(n / K_) * 3 * P_ : p_;
  }
  T* gslot(int n) const {
    if (!tape_forces_) return gtape_;
    return gtape_ + (long long)(K_ ? n % K_ : n) * 3 * M_;
  }

  void ek_fill_u32(uint32_t* x, uint32_t v, long long n) {
    fk::k_fill<uint32_t><<<grid_for(n, kThreads), kThreads, 0, st_>>>(x, v, n);
    IC_LAUNCHED();
  }

  void fill(T* x, T v, long long n) {
    fk::k_fill<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(x, v, n);
    IC_LAUNCHED();
  }
  void copy(const T* a, T* b, long long n) {
    IC_HIP(hipMemcpyAsync(b, a, n * sizeof(T), hipMemcpyDeviceToDevice, st_));
  }

  double sizeT() const { return (double)sizeof(T); }

  // sum over blocks of part[stride * b + k] into scal_[k..k+stride), then to host.
  void reduce_parts(int nblocks, int stride, double* host) {
    fk::k_reduce_parts<<<1, fk::kRedThreads, 0, st_>>>(part_, nblocks, stride, scal_);
    IC_LAUNCHED();
    IC_HIP(hipMemcpyAsync(host, scal_, stride * sizeof(double), hipMemcpyDeviceToHost, st_));
    IC_HIP(hipStreamSynchronize(st_));
  }

  double dot(const T* a, const T* b, long long n) {
    const unsigned g = grid_for(n, fk::kRedThreads, kRedBlocks);
    fk::k_dot<T><<<g, fk::kRedThreads, 0, st_>>>(a, b, part_, n);
    IC_LAUNCHED();
    double r = 0;
    reduce_parts(g, 1, &r);
    return r;
  }

  double dot_diff(const T* g, const T* a, const T* b) {
    const unsigned gr = grid_for(P_, fk::kRedThreads, kRedBlocks);
    fk::k_dot_diff<T><<<gr, fk::kRedThreads, 0, st_>>>(g, a, b, part_, P_);
    IC_LAUNCHED();
    double r = 0;
    reduce_parts(gr, 1, &r);
    return r;
  }

  long long count_nonfinite(const T* x, long long n) {
    const unsigned g = grid_for(n, fk::kRedThreads, kRedBlocks);
    fk::k_count_nonfinite<T><<<g, fk::kRedThreads, 0, st_>>>(x, part_, n);
    IC_LAUNCHED();
    double r = 0;
    reduce_parts(g, 1, &r);
    return (long long)r;
  }

  void scale(const T* x, double alpha, T* y, long long n) {
    fk::k_scale<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(x, static_cast<T>(alpha), y, n);
    IC_LAUNCHED();
  }

  void axpy(const T* a, const T* b, double alpha, T* y, long long n) {
    fk::k_axpy<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(a, b, static_cast<T>(alpha), y, n);
    IC_LAUNCHED();
  }

  // ------------------------------------------------------ block orders
  struct Order {
    unsigned* start;   // nb + 1
    unsigned* istart;  // nb + 1 (istart[nb] = item count)
    uint2* items;
    unsigned nb;
    unsigned max_items;
  };
  Order mesh_order(int n) const {
    return Order{ostart_ + (size_t)n * (nbm_ + 1), oistart_ + (size_t)n * (nbm_ + 1),
                 oitems_ + (size_t)n * mim_, nbm_, mim_};
  }
  Order data_order() const { return Order{dstart_, distart_, ditems_, nbd_, mid_}; }
  unsigned* ids(int n) const { return idtape_ + (size_t)n * P_; }
  // dest(n): slot in order n + 1 of each slot of order n (n = -1: lattice
  // order to order 0); dest(S) maps order S to the data order.
  unsigned* dest(int n) const { return desttape_ + (size_t)(n + 1) * P_; }
  bk::Items items(const Order& o, const unsigned* id) const {
    return bk::Items{o.items, o.start, o.istart + o.nb, id};
  }

  void zero_counts(unsigned nb) { ek_fill_u32(bcount_, 0u, nb); }

  // Scan of the block counts in bcount_ into o, and its work items.
  void build_order(const Order& o) {
    auto sc = timer_.scope("sort_scan", 16.0 * o.nb);
    const unsigned chunks = (o.nb + bk::kScanChunk - 1) / bk::kScanChunk;
    if (chunks > 1024) throw ApiError(IC_ERR_UNSUPPORTED, "too many particle blocks");
    bk::k_scan_sums<<<chunks, 256, 0, st_>>>(bcount_, o.nb, bsums_);
    IC_LAUNCHED();
    bk::k_scan_top<<<1, 1024, 0, st_>>>(bsums_, chunks);
    IC_LAUNCHED();
    bk::k_scan_out<<<chunks, 256, 0, st_>>>(bcount_, o.nb, bsums_, o.start, o.istart);
    IC_LAUNCHED();
    bk::k_fill_items<<<grid_for(o.nb, 256), 256, 0, st_>>>(o.start, o.istart, o.nb, o.items);
    IC_LAUNCHED();
  }

  // Moves nf state fields to the order o (keys and ranks in bkey_ / brank_).
  void scatter(const Order& o, const bk::Ptrs<T>& src, const bk::MPtrs<T>& dst, int nf,
               const unsigned* ids_src, unsigned* ids_dst, unsigned* dst_slots) {
    auto sc = timer_.scope("sort_scatter", P_ * (2.0 * nf * sizeT() + 20.0));
    bk::k_scatter<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
        bkey_, brank_, o.start, src, dst, nf, ids_src, ids_dst, dst_slots, P_);
    IC_LAUNCHED();
  }

  // The ids alone to the order o (keys and ranks in bkey_ / brank_; ids_src
  // null means the lattice order), the destinations to dst_slots, and pinv_
  // = o's slots to the source order's.
  void scatter_ids(const Order& o, const unsigned* ids_src, unsigned* ids_dst,
                   unsigned* dst_slots) {
    auto sc = timer_.scope("sort_scatter_ids", P_ * 24.0);
    bk::k_scatter_ids<<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
        bkey_, brank_, o.start, ids_src, ids_dst, dst_slots, pinv_, P_);
    IC_LAUNCHED();
  }

  // Keys and ranks of displacements d (lattice order) on grid g.
  void keys_lattice(const T* d, const pk::Grid<T>& g, const bk::Layout& L, unsigned nb) {
    zero_counts(nb);
    auto sc = timer_.scope("sort_keys", P_ * (3.0 * sizeT() + 8.0));
    bk::k_keys<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
        d, nullptr, P_, lp_, g, L, bcount_, bkey_, brank_);
    IC_LAUNCHED();
  }

  // First pass of a paint of order o into nf fields and their z halo: zero
  // what no single work item stores (fields and zh need no fill of their own).
  void zero_unowned(const Order& o, const bk::Layout& L, int nf, const bk::MPtrs<T>& dst, T* zh) {
    const long long nb = 1ll << (3 * L.lnb);
    bk::k_zero_unowned<T><<<grid_for(nb * 64, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
        o.istart, L, nf, dst, zh);
    IC_LAUNCHED();
  }

  // Second pass of a paint of order o: the x/y halo staging added along the
  // grid rows through the blocks' lowest x or y layers, for nf fields.
  void halo_rows(const Order& o, const bk::Layout& L, int nf, const bk::MPtrs<T>& dst) {
    const long long waves = bk::face_waves(L);
    const double cells = (double)(waves / 2) * (64 + 56);
    auto sc = timer_.scope("halo_rows", (double)o.max_items * nf * bk::kHaloXY * sizeT() +
                                            2.0 * nf * cells * sizeT());
    const unsigned grid = grid_for(waves * 64, bk::kThreads, 1u << 30);
    if (nf == 3)
      bk::k_halo_rows<T, 3><<<grid, bk::kThreads, 0, st_>>>(hstage_, o.istart, L, dst);
    else
      bk::k_halo_rows<T, 1><<<grid, bk::kThreads, 0, st_>>>(hstage_, o.istart, L, dst);
    IC_LAUNCHED();
  }

  // ------------------------------------------------- deterministic mode
  // The paints accumulate in 64-bit fixed point with one scale per paint and
  // add their windows into det64_ with integer atomics, so a paint's result
  // depends neither on the atomics' order nor on which particles share a
  // work item; the fields are then converted and left complete (their z
  // halo buffers zeroed, no x/y halo pass).
  bk::DetOut det_out(const double* vmax, long long ncells) const {
    return bk::DetOut{det64_, detzh_, detstage_, vmax, ncells, 3 * lp_};
  }
  bk::MPtrs<unsigned long long> det_fields(long long ncells) const {
    return bk::MPtrs<unsigned long long>{{det64_, det64_ + ncells, det64_ + 2 * ncells}};
  }
  // Before a deterministic paint of order o: the integer cells and z-halo
  // entries that no single work item stores.
  void det_zero_unowned(const Order& o, const bk::Layout& L, int nf, long long ncells) {
    const long long nb = 1ll << (3 * L.lnb);
    bk::k_zero_unowned<unsigned long long>
        <<<grid_for(nb * 64, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
            o.istart, L, nf, det_fields(ncells), detzh_);
    IC_LAUNCHED();
  }
  // After it: the x/y halo staging into the integer cells, then the fields.
  void det_finish(const Order& o, const bk::Layout& L, const double* vmax, T coef, int nf,
                  long long ncells, const bk::MPtrs<T>& out) {
    const unsigned grid = grid_for(bk::face_waves(L) * 64, bk::kThreads, 1u << 30);
    if (nf == 3)
      bk::k_halo_rows<unsigned long long, 3>
          <<<grid, bk::kThreads, 0, st_>>>(detstage_, o.istart, L, det_fields(ncells));
    else
      bk::k_halo_rows<unsigned long long, 1>
          <<<grid, bk::kThreads, 0, st_>>>(detstage_, o.istart, L, det_fields(ncells));
    IC_LAUNCHED();
    bk::k_det_to_field<T><<<grid_for(ncells, bk::kThreads), bk::kThreads, 0, st_>>>(
        det64_, detzh_, nf, ncells, L.lm, vmax, coef, 3 * lp_, out);
    IC_LAUNCHED();
  }
  // *out = max |x_i| over n values.
  void absmax(const T* x, long long n, double* out) {
    const unsigned g = grid_for(n, fk::kRedThreads, kRedBlocks);
    fk::k_absmax_parts<T><<<g, fk::kRedThreads, 0, st_>>>(x, n, part_);
    IC_LAUNCHED();
    fk::k_max_parts<<<1, fk::kRedThreads, 0, st_>>>(part_, g, out);
    IC_LAUNCHED();
  }

  // rho = CIC density of the state in order o (positions d, ids id), its
  // z halo left in zh (ncells / 8 values) for the consumer; every cell of
  // rho and zh is written here.  With gsrc the positions are read as
  // d[gsrc[a]] (left in the previous order) and stored in order o to dcopy.
  void paint(const T* d, const Order& o, const unsigned* id, const pk::Grid<T>& g,
             const bk::Layout& L, T* rho, T* zh, long long ncells,
             const unsigned* gsrc = nullptr, T* dcopy = nullptr) {
    const double bytes = P_ * ((gsrc ? 6.0 : 3.0) * sizeT() + (gsrc ? 8.0 : 4.0)) +
                         2.0 * ncells * sizeT();
    if (det_) {
      det_zero_unowned(o, L, 1, ncells);
      {
        auto sc = timer_.scope("cic_paint", bytes);
        bk::k_paint_b<T, true><<<o.max_items + 8, bk::kThreads, 0, st_>>>(
            d, gsrc, dcopy, P_, lp_, g, L, items(o, id), rho, zh, hstage_,
            det_out(nullptr, ncells));
        IC_LAUNCHED();
      }
      det_finish(o, L, nullptr, T(1), 1, ncells, bk::MPtrs<T>{{rho}});
      fill(zh, T(0), ncells / kZHalo);  // the halo is in rho already
      return;
    }
    zero_unowned(o, L, 1, bk::MPtrs<T>{{rho}}, zh);
    {
      auto sc = timer_.scope("cic_paint", bytes);
      bk::k_paint_b<T, false><<<o.max_items + 8, bk::kThreads, 0, st_>>>(
          d, gsrc, dcopy, P_, lp_, g, L, items(o, id), rho, zh, hstage_, bk::DetOut{});
      IC_LAUNCHED();
    }
    halo_rows(o, L, 1, bk::MPtrs<T>{{rho}});
  }

  // cell (x, y, 8 k) of rho += zh[(x, y, k)]: a paint's z halo into the
  // field, for the callers that read the field itself.
  void add_zh(T* rho, const T* zh, long long ncells, int lg) {
    const long long nz = ncells / kZHalo;
    bk::k_add_zh<T><<<grid_for(nz, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(rho, zh, lg,
                                                                                   nz);
    IC_LAUNCHED();
  }

  // rho = CIC density of displacements d given in lattice order (sorted into
  // the scratch order o first; tmpd_ receives the sorted positions); with
  // complete = false the z halo stays in zh_ for a consumer that adds it.
  void paint_lattice(const T* d, int grid, T* rho, bool complete = true) {
    const pk::Grid<T> g = grid ? gmesh() : gdata();
    const bk::Layout& L = grid ? Lm_ : Ld_;
    const Order o = grid ? mesh_order(0) : data_order();
    const long long ncells = grid ? M_ : P_;
    keys_lattice(d, g, L, o.nb);
    build_order(o);
    scatter(o, bk::Ptrs<T>{{d, d + P_, d + 2 * P_}},
            bk::MPtrs<T>{{tmpd_, tmpd_ + P_, tmpd_ + 2 * P_}}, 3, nullptr, dids_, dest(-1));
    paint(tmpd_, o, dids_, g, L, rho, zh_, ncells);
    if (complete) add_zh(rho, zh_, ncells, L.lm);
  }

  // ------------------------------------------------------ k-space chains
  static MulSpec spec(int kinds, int a, int b, double scale) {
    MulSpec s;
    s.kinds = kinds;
    s.ga = a;
    s.ha = a;
    s.hb = b;
    s.scale = scale;
    return s;
  }

  // outs[j] = Op_{spec_j}[alpha (a + zh) + beta b] on the chosen grid (zh:
  // a paint's z halo, nullable).
  void chain_scatter(int grid, const T* a, T alpha, const T* b, T beta, T* const* outs,
                     const MulSpec* specs, int m, const T* zh = nullptr) {
    auto f = fa(grid);
    const long long H = grid ? Hm_ : Hp_;
    const double U = (double)(grid ? M_ : P_) * sizeT();
    const double Hb = half_spectrum_bytes(f.n);
    cx<T>* S0 = pool_;
    cx<T>* So[kMaxMul];
    for (int j = 0; j < m; ++j) So[j] = pool_ + (j + 1) * H;
    r2c_zy(f, a, alpha, b, beta, S0, zh, U, Hb);
    {
      auto sc = timer_.scope("fft_x_scatter", (1 + m) * Hb);
      fft_x_scatter<T>(f, S0, So, specs, m);
    }
    for (int j = 0; j < m; ++j) c2r_yz(f, So[j], outs[j], nullptr, T(0), U, Hb);
  }

  // The z and y passes of a chain: fused into one pass where the grid allows
  // (the chains' spectra are those of real fields), else two.
  void r2c_zy(const FftArgs<T>& f, const T* a, T alpha, const T* b, T beta, cx<T>* S,
              const T* zh, double U, double Hb) {
    if (fft_zy_fused<T>(f.n)) {
      auto sc = timer_.scope("fft_r2c_zy", (b ? 2 : 1) * U + Hb);
      fft_r2c_zy<T>(f, a, alpha, b, beta, S, zh);
      return;
    }
    {
      auto sc = timer_.scope("fft_r2c_z", (b ? 2 : 1) * U + Hb);
      fft_r2c_z<T>(f, a, alpha, b, beta, S, zh);
    }
    auto sc = timer_.scope("fft_y", 2 * Hb);
    fft_y<T>(f, S, true);
  }
  void c2r_yz(const FftArgs<T>& f, cx<T>* S, T* out, const T* aux, T beta_aux, double U,
              double Hb) {
    if (!aux && fft_zy_fused<T>(f.n)) {
      auto sc = timer_.scope("fft_c2r_yz", Hb + U);
      fft_c2r_yz<T>(f, S, out);
      return;
    }
    {
      auto sc = timer_.scope("fft_y", 2 * Hb);
      fft_y<T>(f, S, false);
    }
    auto sc = timer_.scope("fft_c2r_z", Hb + (aux ? 2 : 1) * U);
    fft_c2r_z<T>(f, S, out, T(1), aux, beta_aux);
  }

  struct GIn {
    const T* a;
    T alpha;
    const T* b;
    T beta;
    const T* zh;  // a paint's z halo added to a (nullable)
  };

  // out = sum_j Op_{spec_j}[alpha_j a_j + beta_j b_j] + beta_aux aux.
  void chain_gather(int grid, const GIn* ins, const MulSpec* specs, int m, T* out, const T* aux,
                    T beta_aux) {
    auto f = fa(grid);
    const long long H = grid ? Hm_ : Hp_;
    const double U = (double)(grid ? M_ : P_) * sizeT();
    const double Hb = half_spectrum_bytes(f.n);
    const cx<T>* Si[kMaxMul];
    for (int j = 0; j < m; ++j) {
      cx<T>* Sj = pool_ + j * H;
      r2c_zy(f, ins[j].a, ins[j].alpha, ins[j].b, ins[j].beta, Sj, ins[j].zh, U, Hb);
      Si[j] = Sj;
    }
    {
      auto sc = timer_.scope("fft_x_gather", (1 + m) * Hb);
      fft_x_gather<T>(f, Si, specs, m, pool_);
    }
    c2r_yz(f, pool_, out, aux, beta_aux, U, Hb);
  }

  // -------------------------------------------------------------- forward
  // 2LPT from white noise in lattice order: Psi1 -> d0, Psi2 -> p0, then
  // assembled into the displacement d0 and momentum p0 at a_init.
  void lpt(const T* s, T* d0, T* p0) {
    const double inv = 1.0 / (double)P_;
    MulSpec sp[9] = {spec(MUL_WHITE | MUL_GRAD, 0, 0, inv), spec(MUL_WHITE | MUL_GRAD, 1, 0, inv),
                     spec(MUL_WHITE | MUL_GRAD, 2, 0, inv), spec(MUL_WHITE | MUL_HESS, 0, 0, inv),
                     spec(MUL_WHITE | MUL_HESS, 1, 1, inv), spec(MUL_WHITE | MUL_HESS, 2, 2, inv),
                     spec(MUL_WHITE | MUL_HESS, 0, 1, inv), spec(MUL_WHITE | MUL_HESS, 0, 2, inv),
                     spec(MUL_WHITE | MUL_HESS, 1, 2, inv)};
    T* outs[9] = {d0, d0 + P_, d0 + 2 * P_, phi_, phi_ + P_, phi_ + 2 * P_,
                  phi_ + 3 * P_, phi_ + 4 * P_, phi_ + 5 * P_};
    chain_scatter(0, s, T(1), nullptr, T(0), outs, sp, 9);
    {
      auto sc = timer_.scope("lpt_mu2", 7.0 * P_ * sizeT());
      fk::k_mu2<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(phi_, mu_, P_);
      IC_LAUNCHED();
    }
    MulSpec sp2[3] = {spec(MUL_GRAD, 0, 0, -inv), spec(MUL_GRAD, 1, 0, -inv),
                      spec(MUL_GRAD, 2, 0, -inv)};
    T* outs2[3] = {p0, p0 + P_, p0 + 2 * P_};
    chain_scatter(0, mu_, T(1), nullptr, T(0), outs2, sp2, 3);
    const double a2E = prob_.a_init * prob_.a_init * co_.E_init;
    auto sc = timer_.scope("lpt_assemble", 12.0 * P_ * sizeT());
    fk::k_lpt_assemble<T><<<grid_for(3 * P_, kThreads), kThreads, 0, st_>>>(
        d0, p0, static_cast<T>(co_.D1_init), static_cast<T>(co_.D2_init),
        static_cast<T>(a2E * co_.f1_init * co_.D1_init),
        static_cast<T>(a2E * co_.f2_init * co_.D2_init), 3 * P_);
    IC_LAUNCHED();
  }

  // g = -grad lap^-1 (rho / nbar - 1) on the mesh (the -1 only touches k = 0).
  void force_from_density(T* g) {
    const double nbar = (double)P_ / (double)M_;  // particles per mesh cell
    const double sc = 1.0 / (nbar * (double)M_);
    MulSpec sp[3] = {spec(MUL_GRAD, 0, 0, sc), spec(MUL_GRAD, 1, 0, sc), spec(MUL_GRAD, 2, 0, sc)};
    T* outs[3] = {g, g + M_, g + 2 * M_};
    chain_scatter(1, rhom_, T(1), nullptr, T(0), outs, sp, 3, zh_);
  }

  // Force meshes of the state d_n (order n).  With gsrc the positions are
  // still in the previous order in tmpd_ (gsrc: order n's slots to that
  // order's); the paint reads them through gsrc and stores d_n in its slot.
  void force_mesh(int n, T* g, const unsigned* gsrc = nullptr) {
    if (gsrc)
      paint(tmpd_, mesh_order(n), ids(n), gmesh(), Lm_, rhom_, zh_, M_, gsrc, dslot(n));
    else
      paint(dslot(n), mesh_order(n), ids(n), gmesh(), Lm_, rhom_, zh_, M_);
    force_from_density(g);
  }

  // Whether state m must be complete in its own order after the forward's
  // sort (positions and momenta in their slots): the checkpoints and the
  // lightcone snapshots.  The other states leave the new positions and
  // momenta where the step (or the 2LPT) wrote them and move only the ids:
  // the paint stores the positions in the new order as it reads them, and
  // the next step (or the last kick) reads the momenta through the new
  // order's map back.
  bool state_complete(int m) const { return (K_ && m % K_ == 0) || snapshot_index(m) >= 0; }

  // Forward model.  The 2LPT state is sorted into block order 0; every
  // step reads the forces of its order, kicks and drifts, and sorts the new
  // state into the next order (tapes: d_n, ids and dest per order; see
  // state_complete for which states move positions and momenta in the sort
  // and which only their ids); the last kick ends in order S, which the
  // data paint re-sorts on the data grid.
  void run_forward(const T* s) {
    lpt(s, tmpd_, tmpp_);
    keys_lattice(tmpd_, gmesh(), Lm_, nbm_);
    build_order(mesh_order(0));
    // momenta of state n: pin, in order n or, with pinv, in order n - 1 (the
    // lattice order for n = 0)
    const T* pin = pslot(0);
    const unsigned* pinv = nullptr;
    if (state_complete(0)) {
      scatter(mesh_order(0), state_ptrs(tmpd_, tmpp_), state_mptrs(dslot(0), pslot(0)), 6,
              nullptr, ids(0), dest(-1));
      force_mesh(0, gslot(0));
    } else {
      scatter_ids(mesh_order(0), nullptr, ids(0), dest(-1));
      force_mesh(0, gslot(0), pinv_);
      pin = tmpp_;
      pinv = pinv_;
    }
    for (int n = 0; n < S_; ++n) {
      zero_counts(nbm_);
      const bool complete = state_complete(n + 1);
      // the new momenta go to a buffer the step does not read, and that a
      // complete sort can move into pslot(n + 1) (never tmpp_ or pbar2_)
      T* pout = pin == tmpp_ ? pbar2_ : tmpp_;
      step(n, true, pin, pinv, pout);
      build_order(mesh_order(n + 1));
      if (complete) {
        scatter(mesh_order(n + 1), state_ptrs(tmpd_, pout),
                state_mptrs(dslot(n + 1), pslot(n + 1)), 6, ids(n), ids(n + 1), dest(n));
        force_mesh(n + 1, gslot(n + 1));
        pin = pslot(n + 1);
        pinv = nullptr;
      } else {
        scatter_ids(mesh_order(n + 1), ids(n), ids(n + 1), dest(n));
        force_mesh(n + 1, gslot(n + 1), pinv_);
        pin = pout;
        pinv = pinv_;
      }
      const int j = snapshot_index(n + 1);
      if (j >= 0) {
        // state n + 1 synchronised: p_{n+1/2} + K2_n F(d_{n+1})
        auto sc = timer_.scope("lc_snapshot", P_ * (12.0 * sizeT() + 4.0) + 3.0 * M_ * sizeT());
        bk::k_snapshot_b<T><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
            dslot(n + 1), pslot(n + 1), gslot(n + 1), M_, static_cast<T>(co_.K2[n]), P_, lp_,
            gmesh(), Lm_, items(mesh_order(n + 1), ids(n + 1)), snap_ + (size_t)j * 6 * P_);
        IC_LAUNCHED();
      }
    }
    seg_ = K_ ? S_ - S_ % K_ : 0;
    zero_counts(nbd_);
    {
      auto sc = timer_.scope("final_kick", P_ * (9.0 * sizeT() + 12.0) + 3.0 * M_ * sizeT());
      // the final momenta go to pslot(S) in order S (in place when state S
      // is complete; else pin, in tmpp_ or pbar2_, is read through pinv)
      bk::k_final_b<T><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
          dslot(S_), pin, pinv, pslot(S_), gslot(S_), M_, static_cast<T>(co_.kick[S_]), P_, lp_,
          gmesh(), Lm_, items(mesh_order(S_), ids(S_)), rsd(), gdata(), Ld_, bcount_, bkey_,
          brank_);
      IC_LAUNCHED();
    }
    const T* fd = dslot(S_);
    const T* fp = pslot(S_);
    if (lc_on_) {
      // snapshot slots of the final order, then the lightcone state in order
      // S (tmpd_, tmpp_); its redshift-space displacement (dbar2_, free in the
      // forward) keys the data order
      for (size_t j = 0; j < lc_steps_.size(); ++j) {
        const int m = lc_steps_[j];
        auto sc = timer_.scope("lc_slots", P_ * (4.0 * (S_ - m) + 8.0));
        lk::k_snapshot_slots<<<grid_for(P_, kThreads), kThreads, 0, st_>>>(
            dest(m), S_ - m, snapinv_ + j * P_, P_);
        IC_LAUNCHED();
      }
      {
        auto sc = timer_.scope("lc_crossing",
                               P_ * ((6.0 * lc_steps_.size() + 15.0) * sizeT() +
                                     4.0 * (lc_steps_.size() + 1)));
        IC_LK_LAUNCH(k_lightcone, T, lcgeo_, grid_for(P_, kThreads), kThreads, st_, dslot(S_),
                     pslot(S_), ids(S_), snapinv_, snap_, lcgeo_, rsd(), tmpd_, tmpp_, dbar2_,
                     P_, lp_);
        IC_LAUNCHED();
      }
      zero_counts(nbd_);
      auto sc = timer_.scope("sort_keys", P_ * (3.0 * sizeT() + 12.0));
      bk::k_keys<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
          dbar2_, ids(S_), P_, lp_, gdata(), Ld_, bcount_, bkey_, brank_);
      IC_LAUNCHED();
      fd = tmpd_;
      fp = tmpp_;
    }
    build_order(data_order());
    scatter(data_order(), state_ptrs(fd, fp), state_mptrs(dsd_, psd_), 6, ids(S_), dids_,
            dest(S_));
    if (det_) {
      det_zero_unowned(data_order(), Ld_, 1, P_);
      {
        auto sc = timer_.scope("data_paint", P_ * (8.0 * sizeT() + 4.0) + 2.0 * P_ * sizeT());
        bk::k_data_paint_b<T, true><<<bk::item_grid(Ld_, P_), bk::kThreads, 0, st_>>>(
            dsd_, psd_, P_, lp_, rsd(), gdata(), Ld_, items(data_order(), dids_), rhod_, zhd_,
            hstage_, det_out(nullptr, P_));
        IC_LAUNCHED();
      }
      det_finish(data_order(), Ld_, nullptr, T(1), 1, P_, bk::MPtrs<T>{{rhod_}});
      fill(zhd_, T(0), P_ / kZHalo);  // the halo is in rhod_ already
      return;
    }
    zero_unowned(data_order(), Ld_, 1, bk::MPtrs<T>{{rhod_}}, zhd_);
    {
      auto sc = timer_.scope("data_paint", P_ * (8.0 * sizeT() + 4.0) + 2.0 * P_ * sizeT());
      bk::k_data_paint_b<T, false><<<bk::item_grid(Ld_, P_), bk::kThreads, 0, st_>>>(
          dsd_, psd_, P_, lp_, rsd(), gdata(), Ld_, items(data_order(), dids_), rhod_, zhd_,
          hstage_, bk::DetOut{});
      IC_LAUNCHED();
    }
    halo_rows(data_order(), Ld_, 1, bk::MPtrs<T>{{rhod_}});  // z halo: in zhd_, read by the loss
  }

  // Step n: readout of the forces at d_n, kick, drift into (tmpd_, pout) in
  // order n, with the block keys and ranks of the new positions when keyed.
  // The momenta are read from pin, through pinv when they were left in the
  // previous order.
  void step(int n, bool keyed, const T* pin, const unsigned* pinv, T* pout) {
    auto sc = timer_.scope(keyed ? "pm_step" : "pm_step_replay",
                           P_ * (12.0 * sizeT() + (pinv ? 16.0 : 12.0)) + 3.0 * M_ * sizeT());
    bk::k_step_b<T><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
        dslot(n), pin, pinv, gslot(n), M_, static_cast<T>(co_.kick[n]),
        static_cast<T>(co_.Dr[n]), P_, lp_, gmesh(), Lm_, items(mesh_order(n), ids(n)), tmpd_,
        pout, keyed ? bcount_ : nullptr, bkey_, brank_);
    IC_LAUNCHED();
  }

  // Puts the states of the segment holding state n back in their slots:
  // from checkpoint c = K floor(n / K), the steps c .. c + K - 2 run again in
  // the orders the forward recorded (each new state goes to the next order
  // through that step's recorded destinations, so ids and orders stay the
  // ones the adjoint carries its cotangents through).  With taped forces
  // the segment's force meshes are rebuilt too.
  void restore_segment(int n) {
    if (!K_) return;
    const int c = n - n % K_;
    if (c == seg_) return;
    const int last = std::min(c + K_ - 1, S_);
    for (int j = c; j < last; ++j) {
      force_mesh(j, gslot(j));
      step(j, false, pslot(j), nullptr, tmpp_);
      auto sc = timer_.scope("sort_replay", P_ * (12.0 * sizeT() + 4.0));
      bk::k_to_lattice<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
          dest(j), state_ptrs(tmpd_, tmpp_), state_mptrs(dslot(j + 1), pslot(j + 1)), 6, P_);
      IC_LAUNCHED();
    }
    if (tape_forces_) force_mesh(last, gslot(last));
    seg_ = c;
  }

  // Index of the lightcone snapshot taken at step m, or -1.
  int snapshot_index(int m) const {
    for (size_t j = 0; j < lc_steps_.size(); ++j)
      if (lc_steps_[j] == m) return static_cast<int>(j);
    return -1;
  }

  // Snapshot j's cotangents (in its step's order m) into the sweep:
  // d_bar[t] += cd sd_j, p_bar[t] += cp sp_j with t = to[a], the slot in order
  // m + 1 (to = dest(m)), or t = a in order m itself (to null); d_bar may be
  // null.
  void inject(const unsigned* to, int j, T* db, T cd, T cp) {
    auto sc = timer_.scope("lc_inject", P_ * ((db ? 18.0 : 9.0) * sizeT() + (to ? 4.0 : 0.0)));
    lk::k_inject<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(
        to, snapbar_ + (size_t)j * 6 * P_, db, pbar_, cd, cp, P_);
    IC_LAUNCHED();
  }

  bk::Ptrs<T> state_ptrs(const T* d, const T* p) const {
    return bk::Ptrs<T>{{d, d + P_, d + 2 * P_, p, p + P_, p + 2 * P_}};
  }
  bk::MPtrs<T> state_mptrs(T* d, T* p) const {
    return bk::MPtrs<T>{{d, d + P_, d + 2 * P_, p, p + P_, p + 2 * P_}};
  }

  // Cotangents (dbar_, pbar_) of order 0 brought to the lattice order through
  // dest_slots (buffers swapped with dbar2_, pbar2_).
  void cotangents_back(const unsigned* dest_slots) {
    {
      auto sc = timer_.scope("sort_gather_back", P_ * (12.0 * sizeT() + 4.0));
      bk::k_gather_back<T><<<grid_for(P_, bk::kThreads, 1u << 30), bk::kThreads, 0, st_>>>(
          dest_slots, state_ptrs(dbar_, pbar_), state_mptrs(dbar2_, pbar2_), 6, P_);
      IC_LAUNCHED();
    }
    std::swap(dbar_, dbar2_);
    std::swap(pbar_, pbar2_);
  }

  // Loss terms (and adjoint seed) from the data-grid density of the last forward.
  void observe(const T* s, T* delta, T* lambda, ic_loss_terms* t, bool want_loss) {
    const unsigned g = grid_for(P_, fk::kRedThreads, kRedBlocks);
    {
      auto sc = timer_.scope("loss", 5.0 * P_ * sizeT());
      fk::Obs<T> o;
      o.poisson = prob_.loss_kind == IC_LOSS_POISSON ? 1 : 0;
      o.nbar = static_cast<T>(prob_.nbar);
      o.bias = static_cast<T>(prob_.bias);
      o.r_min = static_cast<T>(prob_.r_min);
      o.alpha = static_cast<T>(prob_.bias_alpha);
      o.delta_th = static_cast<T>(prob_.bias_delta_th);
      o.k = static_cast<T>(prob_.bias_k);
      fk::k_loss<T><<<g, fk::kRedThreads, 0, st_>>>(
          rhod_, want_loss ? counts_ : nullptr, resp_, s, o, want_loss ? seed_ : nullptr, delta,
          lambda, part_, P_, zhd_, lp_);
      IC_LAUNCHED();
    }
    if (!t) return;
    double h[3];
    reduce_parts(g, 3, h);
    t->chi2 = h[0];
    t->prior = h[1];
    t->n_masked = (int64_t)h[2];
    t->loss = 0.5 * h[0] + 0.5 * prob_.prior_weight * h[1];
  }

  // -------------------------------------------------------------- adjoint
  // Reverse sweep from the seed in seed_; out = J^T seed + beta_aux aux.
  void adjoint(T* out, const T* aux, T beta_aux) {
    {
      // cotangents in the data order; step S reads them through dest(S)
      auto sc = timer_.scope("data_adjoint", P_ * (13.0 * sizeT() + 4.0));
      bk::k_data_adjoint_b<T><<<bk::item_grid(Ld_, P_), bk::kThreads, 0, st_>>>(
          dsd_, psd_, P_, lp_, rsd(), gdata(), Ld_, items(data_order(), dids_), seed_, dbar_,
          pbar_);
      IC_LAUNCHED();
    }
    if (lc_on_) {
      // lightcone cotangents: final state in place (data order), the other
      // snapshots into snapbar_ (the final state is still in its slots: no
      // segment has been replayed yet)
      auto sc = timer_.scope("lc_adjoint", P_ * (12.0 * lc_steps_.size() + 16.0) * sizeT());
      IC_LK_LAUNCH(k_lightcone_adjoint, T, lcgeo_, grid_for(P_, kThreads), kThreads, st_,
                   dslot(S_), pslot(S_), ids(S_), snapinv_, dest(S_), snap_, lcgeo_, rsd(), dbar_,
                   pbar_, snapbar_, P_, lp_);
      IC_LAUNCHED();
    }
    // rho_bar = delta_bar / nbar with delta_bar = -sum_j Op_g_j[g_bar_j].
    const double sc_rho = -1.0 / ((double)P_ / (double)M_ * (double)M_);
    for (int n = S_; n >= 0; --n) {
      const T coef = static_cast<T>(co_.kick[n]);
      restore_segment(n);
      T* g = gslot(n);
      if (!tape_forces_) force_mesh(n, g);
      const bk::Items it = items(mesh_order(n), ids(n));
      // a snapshot at step n (d_n, p_n + K2_{n-1} F(d_n)): its d cotangent
      // joins d_bar; its p cotangent enters the kick at d_n as r = K2 / c_n
      // times the kicked momentum's (the paint and readout terms scale with
      // c_n), the rest is added after the step
      const int js = n < S_ ? snapshot_index(n) : -1;
      const double r_snap = js >= 0 ? co_.K2[n - 1] / co_.kick[n] : 0.0;
      if (js >= 0) inject(dest(n), js, dbar_, T(1), static_cast<T>(r_snap));
      const bk::MPtrs<T> gb{{gbar_, gbar_ + M_, gbar_ + 2 * M_}};
      if (det_) {
        absmax(pbar_, 3 * P_, detvmax_);  // the paint's scale: max |p_bar| over all slots
        det_zero_unowned(mesh_order(n), Lm_, 3, M_);
        {
          auto sc = timer_.scope("cic_paint_vec", P_ * (6.0 * sizeT() + 8.0) + 6.0 * M_ * sizeT());
          bk::k_paint_vec_b<T, true><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
              dslot(n), pbar_, coef, P_, lp_, gmesh(), Lm_, it, gbar_, M_, dest(n), zh_, hstage_,
              det_out(detvmax_, M_));
          IC_LAUNCHED();
        }
        det_finish(mesh_order(n), Lm_, detvmax_, coef, 3, M_, gb);
        fill(zh_, T(0), 3 * M_ / kZHalo);  // the halo is in the meshes already
      } else {
        zero_unowned(mesh_order(n), Lm_, 3, gb, zh_);
        {
          auto sc = timer_.scope("cic_paint_vec", P_ * (6.0 * sizeT() + 8.0) + 6.0 * M_ * sizeT());
          bk::k_paint_vec_b<T, false><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
              dslot(n), pbar_, coef, P_, lp_, gmesh(), Lm_, it, gbar_, M_, dest(n), zh_, hstage_,
              bk::DetOut{});
          IC_LAUNCHED();
        }
        halo_rows(mesh_order(n), Lm_, 3, gb);
      }
      const long long zm = M_ / kZHalo;
      GIn ins[3] = {{gbar_, T(1), nullptr, T(0), zh_},
                    {gbar_ + M_, T(1), nullptr, T(0), zh_ + zm},
                    {gbar_ + 2 * M_, T(1), nullptr, T(0), zh_ + 2 * zm}};
      MulSpec sp[3] = {spec(MUL_GRAD, 0, 0, sc_rho), spec(MUL_GRAD, 1, 0, sc_rho),
                       spec(MUL_GRAD, 2, 0, sc_rho)};
      chain_gather(1, ins, sp, 3, rhobar_, nullptr, T(0));
      const T drift = n >= 1 ? static_cast<T>(co_.Dr[n - 1]) : T(0);
      {
        // p_bar and d_bar read from order n + 1 (the data order for n = S)
        // through dest(n), written in order n
        auto sc = timer_.scope("force_adjoint", P_ * (15.0 * sizeT() + 8.0) + 4.0 * M_ * sizeT());
        bk::k_force_adjoint_b<T><<<bk::item_grid(Lm_, P_), bk::kThreads, 0, st_>>>(
            dslot(n), pbar_, dbar_, coef, g, rhobar_, M_, drift, P_, lp_, gmesh(), Lm_, it,
            dest(n), dbar2_, pbar2_);
        IC_LAUNCHED();
      }
      std::swap(dbar_, dbar2_);
      std::swap(pbar_, pbar2_);
      if (js >= 0) inject(nullptr, js, nullptr, T(0), static_cast<T>(1.0 - r_snap));
    }
    // order 0 to the lattice order of the 2LPT adjoint
    cotangents_back(dest(-1));
    // 2LPT and whitening adjoint.
    const double inv = 1.0 / (double)P_;
    const double a2E = prob_.a_init * prob_.a_init * co_.E_init;
    const T c1d = static_cast<T>(co_.D1_init), c1p = static_cast<T>(a2E * co_.f1_init * co_.D1_init);
    const T c2d = static_cast<T>(co_.D2_init), c2p = static_cast<T>(a2E * co_.f2_init * co_.D2_init);
    GIn in2[3];
    MulSpec sp2[3];
    for (int j = 0; j < 3; ++j) {
      in2[j] = {dbar_ + j * P_, c2d, pbar_ + j * P_, c2p};
      sp2[j] = spec(MUL_GRAD, j, 0, inv);
    }
    chain_gather(0, in2, sp2, 3, mu_, nullptr, T(0));
    {
      auto sc = timer_.scope("lpt_phi_bar", 13.0 * P_ * sizeT());
      fk::k_phi_bar<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(phi_, mu_, P_);
      IC_LAUNCHED();
    }
    GIn in9[9];
    MulSpec sp9[9];
    const int ha[6] = {0, 1, 2, 0, 0, 1}, hb[6] = {0, 1, 2, 1, 2, 2};
    for (int j = 0; j < 3; ++j) {
      in9[j] = {dbar_ + j * P_, c1d, pbar_ + j * P_, c1p};
      sp9[j] = spec(MUL_WHITE | MUL_GRAD, j, 0, -inv);
    }
    for (int k = 0; k < 6; ++k) {
      in9[3 + k] = {phi_ + k * P_, T(1), nullptr, T(0)};
      sp9[3 + k] = spec(MUL_WHITE | MUL_HESS, ha[k], hb[k], inv);
    }
    chain_gather(0, in9, sp9, 9, out, aux, beta_aux);
  }

  // Full evaluation: loss terms and gradient into grad.
  void eval(const T* s, T* grad, ic_loss_terms* t) {
    run_forward(s);
    observe(s, nullptr, nullptr, t, true);
    adjoint(grad, s, static_cast<T>(prob_.prior_weight));
  }

  // ------------------------------------------------------------ projection
  // P(x): z-score, reset |z| > s_th to the pass's draws, repeated until a pass
  // resets nothing (the output then has mean 0, std 1 and no extremes, and P
  // is idempotent on it); after kMaxProjectPasses passes with resets, a last
  // z-score without resets keeps the moments exact.  Returns the reset count.
  static constexpr int kMaxProjectPasses = 32;

  int project(const T* x, T* out, uint64_t trial, uint64_t event) {
    const unsigned g = grid_for(P_, fk::kRedThreads, kRedBlocks);
    auto sc = timer_.scope("project_pass", 4.0 * P_ * sizeT());
    int total = 0;
    const T* src = x;
    for (int pass = 0; pass <= kMaxProjectPasses; ++pass) {
      const bool last = pass == kMaxProjectPasses;
      fk::k_dot<T><<<g, fk::kRedThreads, 0, st_>>>(src, nullptr, part_, P_);
      IC_LAUNCHED();
      fk::k_reduce_parts<<<1, fk::kRedThreads, 0, st_>>>(part_, g, 1, scal_);
      IC_LAUNCHED();
      fk::k_centered_sq<T><<<g, fk::kRedThreads, 0, st_>>>(src, scal_, part_, P_);
      IC_LAUNCHED();
      fk::k_reduce_parts<<<1, fk::kRedThreads, 0, st_>>>(part_, g, 1, scal_ + 1);
      IC_LAUNCHED();
      const T th = last ? std::numeric_limits<T>::infinity() : static_cast<T>(prob_.s_th);
      fk::k_project<T><<<g, fk::kRedThreads, 0, st_>>>(src, scal_, scal_ + 1, th,
                                                       trial + 1024ull * pass, event,
                                                       prob_.seed, out, part_, P_);
      IC_LAUNCHED();
      double r = 0;
      reduce_parts(g, 1, &r);
      total += (int)r;
      src = out;
      if (r == 0) break;
    }
    return total;
  }

  // ------------------------------------------------------------------ ROM
  long long rom_real(T* s, uint64_t event);
  long long rom_fourier(T* s, uint64_t event, int32_t* bins_used, bool reim);

  // members
  ic_problem prob_;
  hipStream_t st_;
  Coeffs co_;
  int np_, nm_, S_, lp_, lm_, ratio_;
  long long P_, M_;
  // lightcone: snapshot steps, their states and cotangents, the a(chi) table
  static constexpr int kLcNodes = 1024;
  bool lc_on_ = false;
  std::vector<int> lc_steps_;
  T* snap_ = nullptr;
  T* snapbar_ = nullptr;
  uint32_t* snapinv_ = nullptr;  // snapshot slot of every final slot, per snapshot
  double* lct_ = nullptr;
  lk::LcGeo lcgeo_{};
  int kpp_ = 0, kpm_ = 0;  // stored half-spectrum row pitches (particle grid, mesh)
  long long Hp_, Hm_;      // stored half-spectrum sizes (padded rows)
  long long Hq_;           // half-spectrum modes of the particle grid, n^2 (n/2+1)
  bool tape_forces_;
  int wtab_len_;
  long long rom_len_;
  long long sort_blocks_;
  size_t need_ = 0;
  long long pool_len_ = 0;
  cx<T>* twp_;
  cx<T>* twm_;
  T* wtab_;
  cx<T>* pool_;
  T *phi_, *mu_, *dtape_, *gtape_, *p_, *rhom_, *rhod_, *seed_;
  T* ckp_ = nullptr;   // checkpointed momenta (K_ > 0)
  int K_ = 0;          // checkpoint spacing (0: every state kept)
  int seg_ = -1;       // first state of the segment whose states are in their slots
  T *dbar_, *pbar_, *gbar_, *rhobar_;
  double *part_, *scal_, *lbs_;
  T *hist_S_, *hist_Y_, *dir_, *strial_, *gtrial_;
  uint64_t *keys_, *keys2_;
  uint32_t *vals_, *vals2_, *small_, *shist_, *binc_;
  bk::Layout Lm_{}, Ld_{};  // 8^3-cell blocks of the mesh and of the data grid
  unsigned nbm_ = 0, nbd_ = 0, mim_ = 0, mid_ = 0;
  uint32_t *idtape_, *desttape_, *ostart_, *oistart_, *dstart_, *distart_, *dids_;
  uint2 *oitems_, *ditems_, *bsums_;
  uint32_t *bcount_, *bkey_, *brank_;
  uint32_t* pinv_;  // the newest order's slots to the previous order's
  T* hstage_ = nullptr;
  T* zh_ = nullptr;
  T* zhd_ = nullptr;
  bool det_ = false;                       // deterministic mode
  unsigned long long* det64_ = nullptr;    // its integer paint fields
  unsigned long long* detzh_ = nullptr;    // their z halo
  unsigned long long* detstage_ = nullptr; // their x/y halo staging
  double* detvmax_ = nullptr;              // its cotangent paint's max |p_bar|
  static_assert(bk::kB == kZHalo, "the z halo spacing is the block side");
  T *tmpd_, *tmpp_, *dsd_, *psd_, *dbar2_, *pbar2_;
  T *vbuf_, *tbuf_;
  uint32_t* dbg_idx_[2];
  T* dbg_key_[2];
  uint32_t* dbg_bin_;
  long long dbg_n_[2] = {-1, -1};
  // Host staging of the Fourier-space bin counts and starts; members so that
  // asynchronous copies never outlive their source.
  std::vector<uint32_t> bin_count_ = std::vector<uint32_t>(256, 0);
  std::vector<uint32_t> bin_start_ = std::vector<uint32_t>(128, 0);
  const int32_t* counts_ = nullptr;
  const T* resp_ = nullptr;
  KernelTimer timer_;
  // L-BFGS history: slot ids oldest..newest, their rho = 1/(S.Y), S.Y and Y.Y.
  std::deque<int> hist_;
  std::vector<int> free_slots_;
  double hist_rho_[64] = {}, hist_sy_[64] = {}, hist_yy_[64] = {};
};

}  // namespace ic

#include "engine_ops.h"
