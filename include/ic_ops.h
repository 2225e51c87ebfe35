/*
 * ic_ops.h - single stages of the hot path behind the same context as
 * ic_api.h, for stage-by-stage parity checks and per-kernel timing.  All
 * buffers are device buffers of the context's precision unless stated;
 * conventions (status codes, streams, layouts) are those of ic_api.h.
 */
#ifndef IC_OPS_H
#define IC_OPS_H

#include <stddef.h>
#include <stdint.h>

#include "ic_api.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IC_GRID_PART 0   /* n_part^3 white-noise / particle / data grid */
#define IC_GRID_MESH 1   /* n_mesh^3 particle-mesh force grid */

#define IC_MULT_WHITE 1  /* w(k) = sqrt(P(k) / dq^3), w(0) = 0 (section 2.2.1 item 1) */
#define IC_MULT_GRAD 2   /* i k~_a / k^2: Op[delta] = -grad lap^-1 delta (axis a) */
#define IC_MULT_HESS 4   /* k~_a k~_b / k^2: Op[delta] = d_a d_b lap^-1 delta */

/* Unnormalised forward real DFT of a real cube x (side of the grid) into
 * the half spectrum xk: complex [n][n][n/2+1], interleaved re/im. */
int ic_op_rfft(ic_ctx* ctx, int grid, const void* x, void* xk);

/* Inverse of ic_op_rfft, scaled by 1/n^3 (imaginary parts of the kz = 0
 * and kz = n/2 planes ignored).  xk is left unchanged. */
int ic_op_irfft(ic_ctx* ctx, int grid, const void* xk, void* x);

/* y = Op_m[x] = irfft(m(k) rfft(x)) on the particle grid, m the product of
 * the kinds in kind_bits (WHITE, GRAD along axis_a, HESS along axis_a and
 * axis_b); multipliers vanish at k = 0. */
int ic_op_multiplier(ic_ctx* ctx, int kind_bits, int axis_a, int axis_b,
                     const void* x, void* y);

/* rho(c) = sum_n W(q_n + disp_n - c): cloud-in-cell density of the lattice
 * particles displaced by disp ([3][n_part^3]) on the chosen grid. */
int ic_op_paint(ic_ctx* ctx, int grid, const void* disp, void* rho);

/* Particle-mesh force F_n = sum_c W(x_n - c) g(c), g = -grad lap^-1 delta_m,
 * at x = q + disp; force is [3][n_part^3].  The paint, force chain and
 * readout are the forward model's own kernels (the readout is the step
 * kernel's, with a unit kick from zero momentum and no drift). */
int ic_op_force(ic_ctx* ctx, const void* disp, void* force);

/* 2LPT displacement d0 and momentum p0 at a_init from white noise s
 * (section 2.2.1 items 1-2); both [3][n_part^3]. */
int ic_op_lpt(ic_ctx* ctx, const void* s, void* d0, void* p0);

/* Final particle state of the forward model: displacement and momentum at
 * a_final ([3][n_part^3] each). */
int ic_op_evolve(ic_ctx* ctx, const void* s, void* d_final, void* p_final);

/* Stable descending order of n values (device, context precision): order
 * receives the indices of the largest, next largest, ... (device int32);
 * ties keep index order, -0 equals +0. */
int ic_op_sort_desc(ic_ctx* ctx, const void* values, int64_t n, int32_t* order);

/* Largest n of ic_op_sort_desc_noalloc (2^21 values: a 128^3 field). */
#define IC_NOALLOC_SORT_MAX (1ll << 21)

/* ic_op_sort_desc without a context, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid allocation): the same stable descending order (order[j] =
 * index of the j-th largest of the n values; ties keep index order, -0
 * equals +0), computed by the same kernels, with the sort's keys, indices
 * and histograms in a file-scope device array of 48 MiB that every device
 * running the call holds until the process ends.  precision: IC_F32 or
 * IC_F64 (values: device, of that type); order: device int32[n]; stream: a
 * hipStream_t (NULL = default stream), synchronised once (the NaN check).
 * Allocates nothing.  Calls that overlap on one device share the array and
 * race.  Errors (message in ic_last_error(NULL)): IC_ERR_INVALID_ARG for
 * n < 0 or n > IC_NOALLOC_SORT_MAX, a null buffer or a bad precision;
 * IC_ERR_NONFINITE when a value is NaN (order untouched). */
int ic_op_sort_desc_noalloc(int precision, const void* values, int64_t n, int32_t* order,
                            void* stream);

/* n draws of the counter-based generator (Philox4x64-10, key = seed,
 * counter (j, sub, stream, event) for j = 0..n-1): kind 0 = N(0,1) normals,
 * 1 = Rayleigh with unit mean square.  out: device, context precision. */
int ic_op_philox(ic_ctx* ctx, int kind, uint64_t sub, uint64_t stream, uint64_t event,
                 int64_t n, void* out);

/* Order of the last rank-order matching pass (space 0 = real, 1 = Fourier):
 * for each matched element in descending-rank order, its flat index (into
 * the field, or into the half spectrum; under IC_ROM_FOURIER_REIM the
 * element index 2 f + c of part c (0 = Re, 1 = Im) of half-spectrum mode f),
 * the key it was ranked by and, in Fourier space, its k bin.  Host buffers
 * of capacity cap; *n receives the element count.  Needs a prior
 * ic_project_rankmatch on this context. */
int ic_debug_rom_order(ic_ctx* ctx, int space, int32_t* idx, void* keys, int32_t* bins,
                       int64_t cap, int64_t* n);

/* Host-only (no device work): the FP64 coefficients a context for *p would
 * use, written to out[0..n): D1, f1, D2, f2 and E at a_init, the RSD factor
 * 1/(a_final^2 E), the power-spectrum amplitude A, then Dr_0..Dr_{S-1},
 * K1_0..K1_{S-1}, K2_0..K2_{S-1}.  Needs n >= 7 + 3 n_steps. */
int ic_host_coefficients(const ic_problem* p, double* out, size_t n);

/* Per-kernel timing with HIP events on the context stream: enable != 0
 * starts recording (resetting the totals), 0 stops.  ic_timing_report
 * writes "name count total_ms bytes_per_launch" lines into buf (IC_ERR_
 * INVALID_ARG when len is too small), where bytes_per_launch is the
 * implementation's own count: each buffer a launch reads or writes, once.
 * ic_timing_only starts recording the launches of one kernel name only
 * (kernel: a name the report uses, not NULL), so timed code is otherwise
 * unchanged; ic_timing(ctx, 0) stops it. */
int ic_timing(ic_ctx* ctx, int enable);
int ic_timing_only(ic_ctx* ctx, const char* kernel);
int ic_timing_report(ic_ctx* ctx, char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* IC_OPS_H */
