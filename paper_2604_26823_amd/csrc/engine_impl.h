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
#include "particles.h"
#include "particles_tiled.h"
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
  static constexpr unsigned kRedBlocks = 1024;

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
    tg_ = tk::tile_geom(np_);
    const int m = std::max(1, p.lbfgs_m);
    wtab_len_ = 3 * (np_ / 2) * (np_ / 2) + 1;
    sort_blocks_ = (P_ + sk::kTile - 1) / sk::kTile;

    Carver c(ws);
    twp_ = c.take<cx<T>>(np_);
    twm_ = c.take<cx<T>>(nm_);
    wtab_ = c.take<T>(wtab_len_);
    pool_len_ = std::max(10 * Hp_, 4 * Hm_);
    pool_ = c.take<cx<T>>(pool_len_);
    phi_ = c.take<T>(6 * P_);
    mu_ = c.take<T>(P_);
    dtape_ = c.take<T>((S_ + 1) * 3 * P_);
    gtape_ = c.take<T>((tape_forces_ ? (S_ + 1) : 1) * 3 * M_);
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
    hist_S_ = c.take<T>((size_t)(m + 1) * P_);
    hist_Y_ = c.take<T>((size_t)(m + 1) * P_);
    dir_ = c.take<T>(P_);
    strial_ = c.take<T>(P_);
    gtrial_ = c.take<T>(P_);
    keys_ = c.take<uint64_t>(P_);
    keys2_ = c.take<uint64_t>(P_);
    vals_ = c.take<uint32_t>(P_);
    vals2_ = c.take<uint32_t>(P_);
    small_ = c.take<uint32_t>(P_);
    shist_ = c.take<uint32_t>(sk::kDigits * sort_blocks_);
    vbuf_ = c.take<T>(P_);
    tbuf_ = c.take<T>(P_);
    binc_ = c.take<uint32_t>(256);
    tstat_ = c.take<unsigned long long>(kStatPerKernel * kStatKernels);
    dbg_idx_[0] = c.take<uint32_t>(P_);
    dbg_key_[0] = c.take<T>(P_);
    dbg_idx_[1] = c.take<uint32_t>(Hq_);
    dbg_key_[1] = c.take<T>(Hq_);
    dbg_bin_ = c.take<uint32_t>(Hq_);
    need_ = c.used();
    if (!ws) return;
    if (ws_bytes < need_) throw ApiError(IC_ERR_WORKSPACE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
      throw ApiError(IC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
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
    IC_HIP(hipStreamSynchronize(st_));
  }

  size_t needed() const { return need_; }

  // ------------------------------------------------------------ interface
  void set_stream(hipStream_t s) override {
    st_ = s;
    timer_.set_stream(s);
  }

  void set_observation(const int32_t* counts, const void* response) override {
    if (!counts || !response) throw ApiError(IC_ERR_INVALID_ARG, "null observation buffer");
    counts_ = counts;
    resp_ = static_cast<const T*>(response);
  }

  void forward(const void* s, void* delta, void* lambda, double* loss) override {
    if (!s) throw ApiError(IC_ERR_INVALID_ARG, "s is null");
    if (loss && !counts_) throw ApiError(IC_ERR_STATE, "no observation set");
    if (lambda && !resp_) throw ApiError(IC_ERR_STATE, "no observation set");
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
    ic_loss_terms t{};
    eval(static_cast<const T*>(s), static_cast<T*>(grad), &t);
    if (terms) *terms = t;
    if (!std::isfinite(t.loss)) throw ApiError(IC_ERR_NONFINITE, "loss is not finite");
    if (count_nonfinite(static_cast<const T*>(grad), P_) > 0)
      throw ApiError(IC_ERR_NONFINITE, "gradient is not finite");
  }

  void vjp(const void* s, const void* delta_bar, void* s_bar) override {
    if (!s || !delta_bar || !s_bar) throw ApiError(IC_ERR_INVALID_ARG, "null buffer");
    run_forward(static_cast<const T*>(s));
    copy(static_cast<const T*>(delta_bar), seed_, P_);
    adjoint(static_cast<T*>(s_bar), nullptr, T(0));
  }

  void project_rankmatch(void* sv, uint32_t flags, uint64_t event, int32_t trial,
                         ic_rom_info* info) override {
    if (!sv) throw ApiError(IC_ERR_INVALID_ARG, "s is null");
    T* s = static_cast<T*>(sv);
    ic_rom_info inf{};
    if (flags & (IC_ROM_REAL | IC_ROM_FOURIER)) {
      if (count_nonfinite(s, P_) > 0) throw ApiError(IC_ERR_NONFINITE, "non-finite input to matching");
    }
    if (flags & IC_ROM_REAL) {
      if (!resp_) throw ApiError(IC_ERR_STATE, "real-space matching needs the response field");
      inf.n_real = rom_real(s, event);
    }
    if (flags & IC_ROM_FOURIER) inf.n_fourier = rom_fourier(s, event, &inf.bins_used);
    if (flags & IC_PROJECT) inf.resets = project(s, s, (uint64_t)trial, event);
    if (info) *info = inf;
  }

  void lbfgs_step(void* sv, void* gv, double* loss, int64_t it, ic_lbfgs_info* info) override;

  void lbfgs_reset() override {
    free_slots_.insert(free_slots_.end(), hist_.begin(), hist_.end());
    hist_.clear();
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
    T* r = static_cast<T*>(rho);
    const long long n3 = grid ? M_ : P_;
    fill(r, T(0), n3);
    paint(static_cast<const T*>(disp), grid ? gmesh() : gdata(), r, n3);
  }

  void op_force(const void* disp, void* force) override {
    const T* d = static_cast<const T*>(disp);
    force_mesh(d, gtape_);
    pk::k_readout<T><<<grid_for(P_, kThreads), kThreads, 0, st_>>>(
        d, gtape_, M_, static_cast<T*>(force), P_, lp_, gmesh());
    IC_LAUNCHED();
  }

  void op_lpt(const void* s, void* d0, void* p0) override {
    lpt(static_cast<const T*>(s));
    copy(dtape_, static_cast<T*>(d0), 3 * P_);
    copy(p_, static_cast<T*>(p0), 3 * P_);
  }

  void op_evolve(const void* s, void* d, void* p) override {
    run_forward(static_cast<const T*>(s));
    copy(dslot(S_), static_cast<T*>(d), 3 * P_);
    copy(p_, static_cast<T*>(p), 3 * P_);
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

  void timing(bool enable) override {
    if (enable) {
      ek_fill_u32(reinterpret_cast<uint32_t*>(tstat_), 0u, 2 * kStatPerKernel * kStatKernels);
    }
    timer_.enable(enable);
  }
  void timing_only(const char* kernel) override {
    if (!kernel || !*kernel) throw ApiError(IC_ERR_INVALID_ARG, "kernel name required");
    timer_.enable(true, kernel);
  }
  std::string timing_report() override {
    std::string r = timer_.report();
    std::vector<unsigned long long> cnt(kStatPerKernel * kStatKernels);
    IC_HIP(hipMemcpyAsync(cnt.data(), tstat_, cnt.size() * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st_));
    IC_HIP(hipStreamSynchronize(st_));
    // Rows "tiles_<kernel> windows 0 cells", "tiles_direct_<kernel> tiles 0 0"
    // and "tiles_max_<kernel> cells 0 0".
    for (int k = 0; k < kStatKernels; ++k) {
      unsigned long long v[4] = {0, 0, 0, 0};
      for (int j = 0; j < tk::kStatSlots; ++j) {
        const unsigned long long* s = cnt.data() + k * kStatPerKernel + tk::kStatWords * j;
        for (int q = 0; q < 3; ++q) v[q] += s[q];
        v[3] = std::max(v[3], s[3]);
      }
      const std::string nm = kStatNames[k];
      r += "tiles_" + nm + " " + std::to_string(v[0]) + " 0 " + std::to_string(v[2]) + "\n";
      r += "tiles_direct_" + nm + " " + std::to_string(v[1]) + " 0 0\n";
      r += "tiles_max_" + nm + " " + std::to_string(v[3]) + " 0 0\n";
    }
    return r;
  }

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

  // Window statistics of a tiled kernel (only while every kernel is timed).
  unsigned long long* ovf(int k) const {
    return timer_.all() ? tstat_ + kStatPerKernel * k : nullptr;
  }

  T* dslot(int n) const { return dtape_ + (long long)n * 3 * P_; }
  T* gslot(int n) const { return tape_forces_ ? gtape_ + (long long)n * 3 * M_ : gtape_; }

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

  void axpy(const T* a, const T* b, double alpha, T* y, long long n) {
    fk::k_axpy<T><<<grid_for(n, kThreads), kThreads, 0, st_>>>(a, b, static_cast<T>(alpha), y, n);
    IC_LAUNCHED();
  }

  void paint(const T* d, pk::Grid<T> g, T* rho, long long ncells) {
    auto sc = timer_.scope("cic_paint", (3.0 * P_ + 2.0 * ncells) * sizeT());
    pk::k_paint_t<T><<<tk::tile_count(tg_), tk::kThreads, 0, st_>>>(d, P_, lp_, tg_, g, rho,
                                                                   ovf(0));
    IC_LAUNCHED();
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

  // outs[j] = Op_{spec_j}[alpha a + beta b] on the chosen grid.
  void chain_scatter(int grid, const T* a, T alpha, const T* b, T beta, T* const* outs,
                     const MulSpec* specs, int m) {
    auto f = fa(grid);
    const long long H = grid ? Hm_ : Hp_;
    const double U = (double)(grid ? M_ : P_) * sizeT();
    const double Hb = half_spectrum_bytes(f.n);
    cx<T>* S0 = pool_;
    cx<T>* So[kMaxMul];
    for (int j = 0; j < m; ++j) So[j] = pool_ + (j + 1) * H;
    {
      auto sc = timer_.scope("fft_r2c_z", (b ? 2 : 1) * U + Hb);
      fft_r2c_z<T>(f, a, alpha, b, beta, S0);
    }
    {
      auto sc = timer_.scope("fft_y", 2 * Hb);
      fft_y<T>(f, S0, true);
    }
    {
      auto sc = timer_.scope("fft_x_scatter", (1 + m) * Hb);
      fft_x_scatter<T>(f, S0, So, specs, m);
    }
    for (int j = 0; j < m; ++j) {
      {
        auto sc = timer_.scope("fft_y", 2 * Hb);
        fft_y<T>(f, So[j], false);
      }
      auto sc = timer_.scope("fft_c2r_z", Hb + U);
      fft_c2r_z<T>(f, So[j], outs[j], T(1), nullptr, T(0));
    }
  }

  struct GIn {
    const T* a;
    T alpha;
    const T* b;
    T beta;
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
      {
        auto sc = timer_.scope("fft_r2c_z", (ins[j].b ? 2 : 1) * U + Hb);
        fft_r2c_z<T>(f, ins[j].a, ins[j].alpha, ins[j].b, ins[j].beta, Sj);
      }
      {
        auto sc = timer_.scope("fft_y", 2 * Hb);
        fft_y<T>(f, Sj, true);
      }
      Si[j] = Sj;
    }
    {
      auto sc = timer_.scope("fft_x_gather", (1 + m) * Hb);
      fft_x_gather<T>(f, Si, specs, m, pool_);
    }
    {
      auto sc = timer_.scope("fft_y", 2 * Hb);
      fft_y<T>(f, pool_, false);
    }
    auto sc = timer_.scope("fft_c2r_z", Hb + (aux ? 2 : 1) * U);
    fft_c2r_z<T>(f, pool_, out, T(1), aux, beta_aux);
  }

  // -------------------------------------------------------------- forward
  // 2LPT from white noise: Psi1 -> dslot(0), Psi2 -> p_, then assembled.
  void lpt(const T* s) {
    const double inv = 1.0 / (double)P_;
    MulSpec sp[9] = {spec(MUL_WHITE | MUL_GRAD, 0, 0, inv), spec(MUL_WHITE | MUL_GRAD, 1, 0, inv),
                     spec(MUL_WHITE | MUL_GRAD, 2, 0, inv), spec(MUL_WHITE | MUL_HESS, 0, 0, inv),
                     spec(MUL_WHITE | MUL_HESS, 1, 1, inv), spec(MUL_WHITE | MUL_HESS, 2, 2, inv),
                     spec(MUL_WHITE | MUL_HESS, 0, 1, inv), spec(MUL_WHITE | MUL_HESS, 0, 2, inv),
                     spec(MUL_WHITE | MUL_HESS, 1, 2, inv)};
    T* d0 = dslot(0);
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
    T* outs2[3] = {p_, p_ + P_, p_ + 2 * P_};
    chain_scatter(0, mu_, T(1), nullptr, T(0), outs2, sp2, 3);
    const double a2E = prob_.a_init * prob_.a_init * co_.E_init;
    auto sc = timer_.scope("lpt_assemble", 12.0 * P_ * sizeT());
    fk::k_lpt_assemble<T><<<grid_for(3 * P_, kThreads), kThreads, 0, st_>>>(
        d0, p_, static_cast<T>(co_.D1_init), static_cast<T>(co_.D2_init),
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
    chain_scatter(1, rhom_, T(1), nullptr, T(0), outs, sp, 3);
  }

  void force_mesh(const T* d, T* g) {
    fill(rhom_, T(0), M_);
    paint(d, gmesh(), rhom_, M_);
    force_from_density(g);
  }

  void run_forward(const T* s) {
    lpt(s);
    force_mesh(dslot(0), gslot(0));
    for (int n = 0; n < S_; ++n) {
      fill(rhom_, T(0), M_);
      {
        auto sc = timer_.scope("pm_step", (12.0 * P_ + 5.0 * M_) * sizeT());
        pk::k_pm_step_t<T><<<tk::tile_count(tg_), tk::kThreads, 0, st_>>>(
            dslot(n), p_, gslot(n), M_, static_cast<T>(co_.kick[n]), static_cast<T>(co_.Dr[n]),
            dslot(n + 1), rhom_, P_, lp_, tg_, gmesh(), ovf(1));
        IC_LAUNCHED();
      }
      force_from_density(gslot(n + 1));
    }
    fill(rhod_, T(0), P_);
    auto sc = timer_.scope("final_rsd_paint", (11.0 * P_ + 3.0 * M_) * sizeT());
    pk::k_final_t<T><<<tk::tile_count(tg_), tk::kThreads, 0, st_>>>(
        dslot(S_), p_, gslot(S_), M_, static_cast<T>(co_.kick[S_]), gmesh(), rsd(), gdata(),
        rhod_, P_, lp_, tg_, ovf(2));
    IC_LAUNCHED();
  }

  // Loss terms (and adjoint seed) from the data-grid density of the last forward.
  void observe(const T* s, T* delta, T* lambda, ic_loss_terms* t, bool want_loss) {
    const unsigned g = grid_for(P_, fk::kRedThreads, kRedBlocks);
    {
      auto sc = timer_.scope("loss", 5.0 * P_ * sizeT());
      fk::k_loss<T><<<g, fk::kRedThreads, 0, st_>>>(
          rhod_, want_loss ? counts_ : nullptr, resp_, s, static_cast<T>(prob_.nbar),
          static_cast<T>(prob_.bias), static_cast<T>(prob_.r_min), want_loss ? seed_ : nullptr,
          delta, lambda, part_, P_);
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
      auto sc = timer_.scope("data_adjoint", 13.0 * P_ * sizeT());
      pk::k_data_adjoint_t<T><<<tk::tile_count(tg_), tk::kThreads, 0, st_>>>(
          dslot(S_), p_, rsd(), gdata(), seed_, dbar_, pbar_, P_, lp_, tg_, ovf(3));
      IC_LAUNCHED();
    }
    // rho_bar = delta_bar / nbar with delta_bar = -sum_j Op_g_j[g_bar_j].
    const double sc_rho = -1.0 / ((double)P_ / (double)M_ * (double)M_);
    for (int n = S_; n >= 0; --n) {
      const T coef = static_cast<T>(co_.kick[n]);
      T* g = gslot(n);
      if (!tape_forces_) force_mesh(dslot(n), g);
      fill(gbar_, T(0), 3 * M_);
      {
        auto sc = timer_.scope("cic_paint_vec", (6.0 * P_ + 6.0 * M_) * sizeT());
        pk::k_paint_vec_t<T><<<tk::tile_count(tg_), tk::kThreads, 0, st_>>>(
            dslot(n), pbar_, coef, P_, lp_, tg_, gmesh(), gbar_, M_, ovf(4));
        IC_LAUNCHED();
      }
      GIn ins[3] = {{gbar_, T(1), nullptr, T(0)},
                    {gbar_ + M_, T(1), nullptr, T(0)},
                    {gbar_ + 2 * M_, T(1), nullptr, T(0)}};
      MulSpec sp[3] = {spec(MUL_GRAD, 0, 0, sc_rho), spec(MUL_GRAD, 1, 0, sc_rho),
                       spec(MUL_GRAD, 2, 0, sc_rho)};
      chain_gather(1, ins, sp, 3, rhobar_, nullptr, T(0));
      const T drift = n >= 1 ? static_cast<T>(co_.Dr[n - 1]) : T(0);
      auto sc = timer_.scope("force_adjoint", (15.0 * P_ + 4.0 * M_) * sizeT());
      pk::k_force_adjoint_t<T><<<tk::tile_count(tg_), tk::kThreads, 0, st_>>>(
          dslot(n), pbar_, dbar_, coef, g, rhobar_, M_, drift, P_, lp_, tg_, gmesh(), ovf(5));
      IC_LAUNCHED();
    }
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
  long long rom_fourier(T* s, uint64_t event, int32_t* bins_used);

  // members
  ic_problem prob_;
  hipStream_t st_;
  Coeffs co_;
  int np_, nm_, S_, lp_, lm_, ratio_;
  long long P_, M_;
  int kpp_ = 0, kpm_ = 0;  // stored half-spectrum row pitches (particle grid, mesh)
  long long Hp_, Hm_;      // stored half-spectrum sizes (padded rows)
  long long Hq_;           // half-spectrum modes of the particle grid, n^2 (n/2+1)
  bool tape_forces_;
  tk::TileGeom tg_;
  int wtab_len_;
  long long sort_blocks_;
  size_t need_ = 0;
  long long pool_len_ = 0;
  cx<T>* twp_;
  cx<T>* twm_;
  T* wtab_;
  cx<T>* pool_;
  T *phi_, *mu_, *dtape_, *gtape_, *p_, *rhom_, *rhod_, *seed_;
  T *dbar_, *pbar_, *gbar_, *rhobar_;
  double *part_, *scal_;
  T *hist_S_, *hist_Y_, *dir_, *strial_, *gtrial_;
  uint64_t *keys_, *keys2_;
  uint32_t *vals_, *vals2_, *small_, *shist_, *binc_;
  unsigned long long* tstat_;  // per tiled kernel: tk::kStatSlots groups of 4 counters
  static constexpr int kStatKernels = 6;
  static constexpr int kStatPerKernel = tk::kStatWords * tk::kStatSlots;
  static constexpr const char* kStatNames[kStatKernels] = {
      "paint", "pm_step", "final", "data_adjoint", "paint_vec", "force_adjoint"};
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
