// extern "C" entry points (include/ic_api.h, include/ic_ops.h): argument
// validation, precision dispatch and the translation of exceptions into
// status codes.  No exception or abort crosses the ABI.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/ic_api.h"
#include "../../include/ic_ops.h"
#include "cosmo.h"
#include "engine.h"

struct ic_ctx {
  ic::EngineBase* eng = nullptr;
  int precision = IC_F32;
  std::string err;
};

namespace {

thread_local std::string g_create_error;

int fail(ic_ctx* ctx, int code, const std::string& msg) {
  if (ctx)
    ctx->err = msg;
  else
    g_create_error = msg;
  return code;
}

template <class F>
int guarded(ic_ctx* ctx, F&& f) {
  if (!ctx || !ctx->eng) return fail(ctx, IC_ERR_INVALID_ARG, "null context");
  try {
    f(*ctx->eng);
    return IC_OK;
  } catch (const ic::ApiError& e) {
    return fail(ctx, e.code, e.what());
  } catch (const ic::HipError& e) {
    return fail(ctx, IC_ERR_HIP, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ctx, IC_ERR_INVALID_ARG, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, IC_ERR_INVALID_ARG, e.what());
  }
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

namespace ic {

void noalloc_sort_desc(int precision, const void* values, int64_t n, int32_t* order,
                       hipStream_t st);  // noalloc.hip

void validate_problem(const ic_problem& p) {
  auto bad = [](int code, const char* m) { throw ApiError(code, m); };
  if (!pow2(p.n_part) || p.n_part < 8 || p.n_part > 512)
    bad(IC_ERR_UNSUPPORTED, "n_part must be a power of two in [8, 512]");
  if (!(p.n_mesh == p.n_part || p.n_mesh == 2 * p.n_part) || p.n_mesh > 1024)
    bad(IC_ERR_UNSUPPORTED, "n_mesh must be n_part or 2 n_part and at most 1024");
  if (p.n_steps < 1 || p.n_steps > 1000) bad(IC_ERR_INVALID_ARG, "n_steps must be in [1, 1000]");
  if (!(p.box > 0)) bad(IC_ERR_INVALID_ARG, "box must be positive");
  if (!(p.a_init > 0 && p.a_final > p.a_init && p.a_final <= 10))
    bad(IC_ERR_INVALID_ARG, "need 0 < a_init < a_final");
  if (!(p.omega_m > 0 && p.omega_m <= 1)) bad(IC_ERR_INVALID_ARG, "omega_m must be in (0, 1]");
  if (!(p.h > 0) || !(p.sigma8 > 0)) bad(IC_ERR_INVALID_ARG, "h and sigma8 must be positive");
  if (p.rsd_mode < IC_RSD_NONE || p.rsd_mode > IC_RSD_RADIAL)
    bad(IC_ERR_INVALID_ARG, "unknown rsd_mode");
  if (!(p.nbar > 0)) bad(IC_ERR_INVALID_ARG, "nbar must be positive");
  if (p.lbfgs_m < 1 || p.lbfgs_m > 62) bad(IC_ERR_INVALID_ARG, "lbfgs_m must be in [1, 62]");
  if (p.max_trials < 1) bad(IC_ERR_INVALID_ARG, "max_trials must be >= 1");
  if (!(p.eps_max > 0)) bad(IC_ERR_INVALID_ARG, "eps_max must be positive");
  if (!(p.s_th > 0)) bad(IC_ERR_INVALID_ARG, "s_th must be positive");
  if (p.rom_nbins < 1 || p.rom_nbins > 127) bad(IC_ERR_INVALID_ARG, "rom_nbins must be in [1, 127]");
  if (p.ckpt_every < 0) bad(IC_ERR_INVALID_ARG, "ckpt_every must be >= 0");
  if (p.loss_kind != IC_LOSS_GAUSS && p.loss_kind != IC_LOSS_POISSON)
    bad(IC_ERR_INVALID_ARG, "unknown loss_kind");
  if (p.loss_kind == IC_LOSS_POISSON && !(p.bias_alpha > 0 && p.bias_k > 0))
    bad(IC_ERR_INVALID_ARG, "bias_alpha and bias_k must be positive");
  if (p.deterministic != 0 && p.deterministic != 1)
    bad(IC_ERR_INVALID_ARG, "deterministic must be 0 or 1");
  if (p.lc_n < 0 || p.lc_n > IC_MAX_SNAPSHOTS) bad(IC_ERR_INVALID_ARG, "lc_n must be in [0, 4]");
  if (p.lc_n > 0) {
    if (p.lc_iterations < 1 || p.lc_iterations > 16)
      bad(IC_ERR_INVALID_ARG, "lc_iterations must be in [1, 16]");
    if (std::fabs(p.lc_a[p.lc_n - 1] - p.a_final) > 1e-9)
      bad(IC_ERR_INVALID_ARG, "the last snapshot must be at a_final");
    for (int j = 0; j + 1 < p.lc_n; ++j) {
      if (!(p.lc_a[j] < p.lc_a[j + 1])) bad(IC_ERR_INVALID_ARG, "snapshots must ascend");
      if (snapshot_step(p, p.lc_a[j]) < 0)
        bad(IC_ERR_INVALID_ARG, "snapshots must sit on interior steps a_m, 1 <= m < n_steps");
    }
  }
}

int snapshot_step(const ic_problem& p, double a) {
  const double da = (p.a_final - p.a_init) / p.n_steps;
  const long m = std::lround((a - p.a_init) / da);
  if (m < 1 || m >= p.n_steps || std::fabs(p.a_init + m * da - a) > 1e-9) return -1;
  return static_cast<int>(m);
}

size_t workspace_bytes(const ic_problem& p, int precision) {
  validate_problem(p);
  if (precision == IC_F32) return workspace_bytes_t<float>(p);
  if (precision == IC_F64) return workspace_bytes_t<double>(p);
  throw ApiError(IC_ERR_INVALID_ARG, "precision must be IC_F32 or IC_F64");
}

EngineBase* make_engine(const ic_problem& p, int precision, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  validate_problem(p);
  if (!ws) throw ApiError(IC_ERR_INVALID_ARG, "workspace is null");
  if (precision == IC_F32) return make_engine_t<float>(p, ws, ws_bytes, stream);
  if (precision == IC_F64) return make_engine_t<double>(p, ws, ws_bytes, stream);
  throw ApiError(IC_ERR_INVALID_ARG, "precision must be IC_F32 or IC_F64");
}

}  // namespace ic

extern "C" {

int32_t ic_abi_version(void) { return IC_ABI_VERSION; }

void ic_problem_defaults(ic_problem* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_steps = 10;
  p->rsd_mode = IC_RSD_RADIAL;
  p->a_init = IC_DEFAULT_A_INIT;
  p->a_final = 1.0;
  p->omega_m = 0.3;
  p->h = 0.7;
  p->n_s = 0.96;
  p->sigma8 = 0.8;
  p->bias = 1.5;
  p->nbar = 1.0;
  p->r_min = 1e-3;
  p->prior_weight = 1.0;
  p->lbfgs_m = 10;
  p->max_trials = 30;
  p->eps_max = IC_DEFAULT_EPS_MAX;
  p->armijo_c1 = 1e-4;
  p->s_th = IC_DEFAULT_S_TH;
  p->rom_nbins = IC_DEFAULT_ROM_NBINS;
  p->tape_forces = 1;
  p->ckpt_every = 0;
  p->loss_kind = IC_LOSS_GAUSS;
  p->bias_alpha = IC_DEFAULT_BIAS_ALPHA;
  p->bias_delta_th = IC_DEFAULT_BIAS_DELTA_TH;
  p->bias_k = IC_DEFAULT_BIAS_K;
  p->project_steps = 1;
  p->lc_n = 0;
  p->lc_iterations = IC_DEFAULT_LC_ITERATIONS;
  p->rom_kmin = IC_DEFAULT_ROM_KMIN;
  p->seed = 0;
}

int ic_workspace_size(const ic_problem* p, int precision, size_t* bytes) {
  if (!p || !bytes) return fail(nullptr, IC_ERR_INVALID_ARG, "null argument");
  try {
    *bytes = ic::workspace_bytes(*p, precision);
    return IC_OK;
  } catch (const ic::ApiError& e) {
    return fail(nullptr, e.code, e.what());
  } catch (const std::exception& e) {
    return fail(nullptr, IC_ERR_INVALID_ARG, e.what());
  }
}

int ic_create(const ic_problem* p, int precision, void* ws, size_t ws_bytes, void* stream,
              ic_ctx** out) {
  if (!p || !out) return fail(nullptr, IC_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  try {
    ic_ctx* c = new ic_ctx();
    try {
      c->eng = ic::make_engine(*p, precision, ws, ws_bytes, static_cast<hipStream_t>(stream));
    } catch (...) {
      delete c;
      throw;
    }
    c->precision = precision;
    *out = c;
    return IC_OK;
  } catch (const ic::ApiError& e) {
    return fail(nullptr, e.code, e.what());
  } catch (const ic::HipError& e) {
    return fail(nullptr, IC_ERR_HIP, e.what());
  } catch (const std::exception& e) {
    return fail(nullptr, IC_ERR_INVALID_ARG, e.what());
  }
}

void ic_destroy(ic_ctx* ctx) {
  if (!ctx) return;
  delete ctx->eng;
  delete ctx;
}

const char* ic_last_error(const ic_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int ic_set_stream(ic_ctx* ctx, void* stream) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.set_stream(static_cast<hipStream_t>(stream)); });
}

int ic_set_observation(ic_ctx* ctx, const int32_t* counts, const void* response) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.set_observation(counts, response); });
}

int ic_forward(ic_ctx* ctx, const void* s, void* delta_s, void* lambda, double* loss) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.forward(s, delta_s, lambda, loss); });
}

int ic_loss_and_grad(ic_ctx* ctx, const void* s, void* grad, double* loss,
                     ic_loss_terms* terms) {
  return guarded(ctx, [&](ic::EngineBase& e) {
    ic_loss_terms t{};
    try {
      e.loss_and_grad(s, grad, &t);
    } catch (...) {
      if (loss) *loss = t.loss;
      if (terms) *terms = t;
      throw;
    }
    if (loss) *loss = t.loss;
    if (terms) *terms = t;
  });
}

int ic_vjp(ic_ctx* ctx, const void* s, const void* delta_bar, void* s_bar) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.vjp(s, delta_bar, s_bar); });
}

int ic_project_rankmatch(ic_ctx* ctx, void* s, uint32_t flags, uint64_t event, int32_t trial,
                         ic_rom_info* info) {
  return guarded(ctx,
                 [&](ic::EngineBase& e) { e.project_rankmatch(s, flags, event, trial, info); });
}

int ic_lbfgs_step(ic_ctx* ctx, void* s, void* grad, double* loss, int64_t iteration,
                  ic_lbfgs_info* info) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.lbfgs_step(s, grad, loss, iteration, info); });
}

int ic_lbfgs_reset(ic_ctx* ctx) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.lbfgs_reset(); });
}

int ic_upsample_noise(ic_ctx* high, ic_ctx* low, const void* s_low, void* s_high,
                      uint64_t event) {
  if (!low || !low->eng) return fail(high, IC_ERR_INVALID_ARG, "null coarse context");
  if (high && low->precision != high->precision)
    return fail(high, IC_ERR_INVALID_ARG, "contexts of different precision");
  if (low == high) return fail(high, IC_ERR_INVALID_ARG, "coarse and fine context are the same");
  return guarded(high, [&](ic::EngineBase& e) { e.upsample_from(*low->eng, s_low, s_high, event); });
}

static int check_grid(ic_ctx* ctx, int grid) {
  if (grid != IC_GRID_PART && grid != IC_GRID_MESH)
    return fail(ctx, IC_ERR_INVALID_ARG, "grid must be IC_GRID_PART or IC_GRID_MESH");
  return IC_OK;
}

int ic_op_rfft(ic_ctx* ctx, int grid, const void* x, void* xk) {
  if (int r = check_grid(ctx, grid)) return r;
  if (!x || !xk) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_rfft(grid, x, xk); });
}

int ic_op_irfft(ic_ctx* ctx, int grid, const void* xk, void* x) {
  if (int r = check_grid(ctx, grid)) return r;
  if (!x || !xk) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_irfft(grid, xk, x); });
}

int ic_op_multiplier(ic_ctx* ctx, int kind_bits, int axis_a, int axis_b, const void* x, void* y) {
  if (!x || !y) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  if (kind_bits < 0 || kind_bits > 7) return fail(ctx, IC_ERR_INVALID_ARG, "unknown multiplier");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_multiplier(kind_bits, axis_a, axis_b, x, y); });
}

int ic_op_paint(ic_ctx* ctx, int grid, const void* disp, void* rho) {
  if (int r = check_grid(ctx, grid)) return r;
  if (!disp || !rho) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_paint(grid, disp, rho); });
}

int ic_op_force(ic_ctx* ctx, const void* disp, void* force) {
  if (!disp || !force) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_force(disp, force); });
}

int ic_op_lpt(ic_ctx* ctx, const void* s, void* d0, void* p0) {
  if (!s || !d0 || !p0) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_lpt(s, d0, p0); });
}

int ic_op_evolve(ic_ctx* ctx, const void* s, void* d_final, void* p_final) {
  if (!s || !d_final || !p_final) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_evolve(s, d_final, p_final); });
}

int ic_op_sort_desc(ic_ctx* ctx, const void* values, int64_t n, int32_t* order) {
  if ((!values || !order) && n > 0) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_sort_desc(values, n, order); });
}

int ic_op_philox(ic_ctx* ctx, int kind, uint64_t sub, uint64_t stream, uint64_t event, int64_t n,
                 void* out) {
  if (kind != 0 && kind != 1) return fail(ctx, IC_ERR_INVALID_ARG, "kind must be 0 or 1");
  if (!out && n > 0) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) { e.op_philox(kind, sub, stream, event, n, out); });
}

int ic_debug_rom_order(ic_ctx* ctx, int space, int32_t* idx, void* keys, int32_t* bins,
                       int64_t cap, int64_t* n) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.debug_rom_order(space, idx, keys, bins, cap, n); });
}

int ic_host_coefficients(const ic_problem* p, double* out, size_t n) {
  if (!p || !out) return fail(nullptr, IC_ERR_INVALID_ARG, "null argument");
  try {
    ic::validate_problem(*p);
    const size_t need = 7 + 3 * (size_t)p->n_steps;
    if (n < need) return fail(nullptr, IC_ERR_INVALID_ARG, "output too short");
    ic::CosmoParams cp{p->omega_m, p->h, p->n_s, p->sigma8, p->a_init, p->a_final, p->n_steps};
    ic::Coeffs c = ic::compute_coeffs(cp);
    const double head[7] = {c.D1_init, c.f1_init, c.D2_init, c.f2_init, c.E_init, c.rsd_factor,
                            c.pk_amplitude};
    std::memcpy(out, head, sizeof(head));
    for (int i = 0; i < p->n_steps; ++i) {
      out[7 + i] = c.Dr[i];
      out[7 + p->n_steps + i] = c.K1[i];
      out[7 + 2 * p->n_steps + i] = c.K2[i];
    }
    return IC_OK;
  } catch (const ic::ApiError& e) {
    return fail(nullptr, e.code, e.what());
  } catch (const std::exception& e) {
    return fail(nullptr, IC_ERR_INVALID_ARG, e.what());
  }
}

int ic_timing(ic_ctx* ctx, int enable) {
  return guarded(ctx, [&](ic::EngineBase& e) { e.timing(enable != 0); });
}

int ic_timing_only(ic_ctx* ctx, const char* kernel) {
  if (!kernel) return fail(ctx, IC_ERR_INVALID_ARG, "null kernel name");
  return guarded(ctx, [&](ic::EngineBase& e) { e.timing_only(kernel); });
}

int ic_timing_report(ic_ctx* ctx, char* buf, size_t len) {
  if (!buf || len == 0) return fail(ctx, IC_ERR_INVALID_ARG, "null buffer");
  return guarded(ctx, [&](ic::EngineBase& e) {
    std::string r = e.timing_report();
    if (r.size() + 1 > len) throw ic::ApiError(IC_ERR_INVALID_ARG, "report buffer too small");
    std::memcpy(buf, r.c_str(), r.size() + 1);
  });
}

int ic_op_sort_desc_noalloc(int precision, const void* values, int64_t n, int32_t* order,
                            void* stream) {
  try {
    ic::noalloc_sort_desc(precision, values, n, order, static_cast<hipStream_t>(stream));
    return IC_OK;
  } catch (const ic::ApiError& e) {
    return fail(nullptr, e.code, e.what());
  } catch (const ic::HipError& e) {
    return fail(nullptr, IC_ERR_HIP, e.what());
  } catch (const std::exception& e) {
    return fail(nullptr, IC_ERR_INVALID_ARG, e.what());
  }
}

}  // extern "C"
