// Precision-independent interface of the hot-path engine; one
// implementation per element type (float, double) sits behind it.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/ic_api.h"
#include "common.h"

namespace ic {

struct EngineBase {
  virtual ~EngineBase() = default;
  virtual void set_stream(hipStream_t s) = 0;
  virtual hipStream_t stream() const = 0;
  virtual const ic_problem& problem() const = 0;
  virtual void set_observation(const int32_t* counts, const void* response) = 0;
  virtual void forward(const void* s, void* delta, void* lambda, double* loss) = 0;
  virtual void loss_and_grad(const void* s, void* grad, ic_loss_terms* terms) = 0;
  virtual void vjp(const void* s, const void* delta_bar, void* s_bar) = 0;
  virtual void project_rankmatch(void* s, uint32_t flags, uint64_t event, int32_t trial,
                                 ic_rom_info* info) = 0;
  virtual void lbfgs_step(void* s, void* grad, double* loss, int64_t iteration,
                          ic_lbfgs_info* info) = 0;
  virtual void lbfgs_reset() = 0;
  // Fine white noise from the coarse field s_low of engine low (same precision,
  // half the particle grid side, same box): see ic_upsample_noise.
  virtual void upsample_from(EngineBase& low, const void* s_low, void* s_high,
                             uint64_t event) = 0;
  // single stages
  virtual void op_rfft(int grid, const void* x, void* xk) = 0;
  virtual void op_irfft(int grid, const void* xk, void* x) = 0;
  virtual void op_multiplier(int kinds, int a, int b, const void* x, void* y) = 0;
  virtual void op_paint(int grid, const void* disp, void* rho) = 0;
  virtual void op_force(const void* disp, void* force) = 0;
  virtual void op_lpt(const void* s, void* d0, void* p0) = 0;
  virtual void op_evolve(const void* s, void* d, void* p) = 0;
  virtual void op_sort_desc(const void* values, int64_t n, int32_t* order) = 0;
  virtual void op_philox(int kind, uint64_t sub, uint64_t stream, uint64_t event, int64_t n,
                         void* out) = 0;
  virtual void debug_rom_order(int space, int32_t* idx, void* keys, int32_t* bins, int64_t cap,
                               int64_t* n) = 0;
  virtual void timing(bool enable) = 0;
  virtual void timing_only(const char* kernel) = 0;
  virtual std::string timing_report() = 0;
};

// Workspace bytes for (problem, precision); throws ApiError on bad input.
size_t workspace_bytes(const ic_problem& p, int precision);

// Builds the engine on the caller's workspace.
EngineBase* make_engine(const ic_problem& p, int precision, void* ws, size_t ws_bytes,
                        hipStream_t stream);

// Shape / parameter validation shared by ic_workspace_size and ic_create.
void validate_problem(const ic_problem& p);

// Step m (1 <= m < n_steps) whose scale factor a_m equals a, else -1.
int snapshot_step(const ic_problem& p, double a);

template <typename T>
size_t workspace_bytes_t(const ic_problem& p);
template <typename T>
EngineBase* make_engine_t(const ic_problem& p, void* ws, size_t ws_bytes, hipStream_t stream);

}  // namespace ic
