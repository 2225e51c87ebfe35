/*
 * ic_api.h - C ABI of the MI355X (gfx950) implementation of the MUJICA
 * initial-condition reconstruction hot path (arXiv 2604.26823).
 *
 * The library evaluates the differentiable forward model of paper section
 * 2.2.1 (white noise -> BBKS-shaped linear field -> 2LPT -> FastPM kick-drift-
 * kick particle mesh -> redshift-space distortion -> linear bias and survey
 * response), the masked Gaussian chi^2 plus white-noise prior built on it,
 * the gradient of that loss by a hand-written adjoint, the projection and
 * rank-order matching of section 2.3, and the projected L-BFGS step of
 * section 2.3.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every int-returning call returns IC_OK (0) or a negative IC_ERR_*
 *   code; ic_last_error() then describes the failure.  Nothing aborts or
 *   throws across the ABI.
 * Ownership: the caller allocates every device buffer: fields passed to the
 *   calls and one workspace block of ic_workspace_size() bytes handed to
 *   ic_create().  The library never allocates or frees device memory and
 *   keeps the workspace, observation and stream pointers until ic_destroy(),
 *   so the caller keeps them alive.  Host pointers (loss, info structs,
 *   debug dumps) are written before the call returns.
 * Streams: all device work is enqueued on the hipStream_t given to
 *   ic_create() / ic_set_stream().  Calls that return host values (losses,
 *   info structs, debug dumps) synchronise that stream; the rest are
 *   asynchronous.  A context is not thread-safe.
 * Precision: fixed per context, IC_F32 or IC_F64.  All field buffers have
 *   that element type; losses and optimiser scalars are always double.
 * Layouts: real fields are C-ordered [x][y][z] cubes of side n_part (the
 *   white-noise, particle and data grid) with z fastest.  Particle arrays are
 *   structure-of-arrays [3][n_part^3] in the same lattice order.
 * Shapes: n_part a power of two in [8, 512]; n_mesh = n_part or 2 n_part and
 *   at most 1024; otherwise IC_ERR_UNSUPPORTED.
 */
#ifndef IC_API_H
#define IC_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IC_ABI_VERSION 6

#define IC_OK 0
#define IC_ERR_INVALID_ARG (-1)
#define IC_ERR_UNSUPPORTED (-2)
#define IC_ERR_WORKSPACE (-3)
#define IC_ERR_HIP (-4)
#define IC_ERR_NONFINITE (-5)
#define IC_ERR_LINESEARCH (-6)
#define IC_ERR_STATE (-7)

#define IC_F32 0
#define IC_F64 1

#define IC_RSD_NONE 0
#define IC_RSD_AXIS_Z 1
#define IC_RSD_RADIAL 2

/* flags of ic_project_rankmatch */
#define IC_PROJECT 1u
#define IC_ROM_REAL 2u
#define IC_ROM_FOURIER 4u
/* Second reading of the Fourier-space matching (section 2.3.2, "matching
 * the Fourier modes"): per k bin, the real and imaginary parts of the n
 * matched modes form one set of 2n values matched to 2n draws of N(0, 1/2)
 * instead of the amplitudes to Rayleigh draws.  Excludes IC_ROM_FOURIER. */
#define IC_ROM_FOURIER_REIM 8u

/* Method parameters the paper fixes (section 2.3.1: reset threshold;
 * section 2.3.2: 100 equal-width k bins, modes below k = 0.1 h/Mpc left
 * alone; section 2.2.1 item 2: 2LPT to a = 0.1; appendix B, table 1: the
 * method's maximum line-search step). */
#define IC_DEFAULT_S_TH 10.0
#define IC_DEFAULT_ROM_NBINS 100
#define IC_DEFAULT_ROM_KMIN 0.1
#define IC_DEFAULT_A_INIT 0.1
#define IC_DEFAULT_EPS_MAX 1.0

/* loss_kind */
#define IC_LOSS_GAUSS 0    /* linear bias, masked Gaussian chi^2 (the benchmarked objective) */
#define IC_LOSS_POISSON 1  /* the paper's bias and Poisson likelihood (sections 2.2.1-2.2.2) */

/* The paper's galaxy bias (section 2.2.1, item 4, the power law times a
 * sigmoid): lambda = nbar R (1 + delta)^alpha sigmoid(K (delta - delta_th)). */
#define IC_DEFAULT_BIAS_ALPHA 0.7
#define IC_DEFAULT_BIAS_DELTA_TH 1.2
#define IC_DEFAULT_BIAS_K 3.0

/* Lightcone (section 2.2.1 item 3, appendix A): at most this many snapshots;
 * the paper saves a = 0.8, 0.9, 1.0 and iterates the crossing scale factor
 * three times. */
#define IC_MAX_SNAPSHOTS 4
#define IC_DEFAULT_LC_ITERATIONS 3

/* The reconstruction problem (sections 2.2-2.3).  Lengths in Mpc/h. */
typedef struct ic_problem {
  int32_t n_part;        /* particles per side = white-noise and data grid side */
  int32_t n_mesh;        /* particle-mesh force grid side (n_part or 2 n_part) */
  int32_t n_steps;       /* kick-drift-kick steps, linear in a, >= 1 */
  int32_t rsd_mode;      /* IC_RSD_NONE, IC_RSD_AXIS_Z or IC_RSD_RADIAL */
  double box;            /* periodic box side */
  double a_init;         /* 2LPT start (0.1) */
  double a_final;        /* output epoch (1.0) */
  double omega_m, h, n_s, sigma8;   /* flat LCDM, BBKS transfer function */
  double observer[3];    /* observer position for radial RSD */
  double bias;           /* linear bias b: lambda = nbar R (1 + b delta_s) */
  double nbar;           /* mean galaxies per data cell */
  double r_min;          /* mask M = [R >= r_min] */
  double prior_weight;   /* weight of 1/2 |s|^2 in the loss */
  int32_t lbfgs_m;       /* history pairs (10) */
  int32_t max_trials;    /* line-search trials (30) */
  double eps_max;        /* first trial step (1.0) */
  double armijo_c1;      /* sufficient-decrease constant (1e-4) */
  double s_th;           /* projection reset threshold (10) */
  int32_t rom_nbins;     /* Fourier-space matching bins (100) */
  int32_t tape_forces;   /* 1: keep force meshes for the adjoint; 0: recompute */
  int32_t ckpt_every;    /* K > 0: keep particle states only at steps 0, K, 2K, ...
                            and recompute the steps in between during the adjoint;
                            0: keep every step's state */
  double rom_kmin;       /* smallest matched |k| (0.1 h/Mpc) */
  uint64_t seed;         /* key of the counter-based generator */
  double bias_alpha;     /* IC_LOSS_POISSON: power-law index alpha (0.7) */
  double bias_delta_th;  /* IC_LOSS_POISSON: sigmoid threshold delta_th (1.2) */
  double bias_k;         /* IC_LOSS_POISSON: sigmoid steepness K (3.0) */
  int32_t loss_kind;     /* IC_LOSS_GAUSS or IC_LOSS_POISSON.  Poisson: lambda = nbar R
                            u^alpha sigmoid(K (delta_s - delta_th)) with u = 1 + delta_s
                            floored at 1e-6 (constant below the floor), data term
                            D = -2 sum_M (N log lambda - lambda - log N!); bias unused */
  int32_t project_steps; /* 1: trial points P(s + eps p) (the method, section 2.3.1);
                            0: plain L-BFGS trial points s + eps p (the ablation's
                            baseline, appendix B) */
  int32_t lc_n;          /* lightcone (section 2.2.1 item 3, appendix A): number of
                            snapshots, 0 = off (RSD and data paint at a_final), else
                            1..IC_MAX_SNAPSHOTS */
  int32_t lc_iterations; /* fixed-point iterations of the crossing scale factor (3) */
  double lc_a[4];        /* snapshot scale factors, ascending; lc_a[lc_n-1] = a_final and
                            the others interior steps a_m, 1 <= m < n_steps.  Each
                            particle's displacement and momentum are interpolated
                            linearly in a between the kick-synchronised snapshots; its
                            scale factor a_i = DistToScaleFactor(|x(a_i) - observer|),
                            iterated lc_iterations times from a_final and clamped to
                            [lc_a[0], a_final], sets where it is painted and its RSD
                            factor 1/(a_i^2 E(a_i)).  Distances: box-wrapped positions,
                            flat-cosmology comoving distance with c/H0 = 2997.92458 */
  int32_t deterministic; /* 1: every result is a function of the inputs alone, bit for bit
                            from run to run.  The three cloud-in-cell paints (density,
                            data grid, the adjoint's momentum-cotangent paint) then sum
                            each cell's contributions as 64-bit integers with one
                            power-of-two scale per paint, chosen from the largest
                            contribution so that no sum of n_part^3 of them can
                            overflow; integer sums do not depend on the order in which
                            they are formed; rounding each contribution to that
                            scale (an absolute error of at most 2^-62 n_part^3 times the
                            largest contribution: 2^-38 of it at n_part = 256) is the
                            mode's only numerical change.
                            0 (default): the paints accumulate in the faster per-block
                            order, whose floating-point rounding can differ between runs */
} ic_problem;

typedef struct ic_loss_terms {
  double loss;           /* 1/2 chi2 + 1/2 prior_weight |s|^2 */
  double chi2;           /* data term D over the masked cells: sum (N - lambda)^2 / (nbar R)
                            (IC_LOSS_GAUSS) or -2 log L of the Poisson model (IC_LOSS_POISSON);
                            loss = 1/2 D + 1/2 prior_weight |s|^2 */
  double prior;          /* |s|^2 */
  int64_t n_masked;      /* cells with R >= r_min */
} ic_loss_terms;

typedef struct ic_lbfgs_info {
  double eps;            /* accepted step */
  double gp;             /* g . p of the search direction */
  int32_t trials;        /* line-search trials used */
  int32_t evaluations;   /* loss+gradient evaluations made */
  int32_t stored;        /* 1 if the (S, Y) pair entered the history */
  int32_t history;       /* pairs held after the step */
  int32_t restarted;     /* 1 if the direction was reset to -g */
  int32_t resets;        /* projection resets in the accepted trial */
} ic_lbfgs_info;

typedef struct ic_rom_info {
  int64_t n_real;        /* elements matched in real space */
  int64_t n_fourier;     /* modes matched in Fourier space */
  int32_t resets;        /* projection resets */
  int32_t bins_used;     /* non-empty k bins */
} ic_rom_info;

typedef struct ic_ctx ic_ctx;

/* ABI version (IC_ABI_VERSION). */
int32_t ic_abi_version(void);

/* Fills *p with the defaults above (n_part, n_mesh, box, rsd_mode left 0). */
void ic_problem_defaults(ic_problem* p);

/* Device bytes the workspace of a context for (*p, precision) needs. */
int ic_workspace_size(const ic_problem* p, int precision, size_t* bytes);

/* Validates *p, lays out the caller's workspace (device pointer ws of
 * ws_bytes bytes, 256-byte aligned) and computes the FP64 cosmology
 * coefficients (growth factors, FastPM kick/drift factors of section 2.2.1
 * item 2, whitening multiplier of item 1).  stream: a hipStream_t (NULL =
 * default stream).  *out receives the context. */
int ic_create(const ic_problem* p, int precision, void* ws, size_t ws_bytes,
              void* stream, ic_ctx** out);

/* Releases the context (host memory only; device buffers stay the caller's). */
void ic_destroy(ic_ctx* ctx);

/* Description of the last failure on ctx (or of the last failed ic_create
 * when ctx is NULL). */
const char* ic_last_error(const ic_ctx* ctx);

/* Changes the stream later calls enqueue on. */
int ic_set_stream(ic_ctx* ctx, void* stream);

/* Observation of section 2.2.1 items 4-5 and 2.2.2: galaxy counts N
 * (int32, device, n_part^3) and survey response R (device, context
 * precision, n_part^3).  Mask M = [R >= r_min]; variance nbar R.  The
 * pointers are kept; the caller keeps the buffers alive and unchanged. */
int ic_set_observation(ic_ctx* ctx, const int32_t* counts, const void* response);

/* Forward model s -> delta_s (section 2.2.1).  s: device, n_part^3.
 * delta_s, lambda: optional device outputs (n_part^3, NULL to skip).
 * loss: optional host output (needs an observation).  Returns
 * IC_ERR_NONFINITE, before any particle moves, when s holds a NaN or inf. */
int ic_forward(ic_ctx* ctx, const void* s, void* delta_s, void* lambda, double* loss);

/* L(s) = 1/2 chi^2 + 1/2 prior_weight |s|^2 and its gradient (device,
 * n_part^3) by the hand-written adjoint of the forward model.  terms is
 * optional.  Returns IC_ERR_NONFINITE when s (checked first), L or the
 * gradient is not finite. */
int ic_loss_and_grad(ic_ctx* ctx, const void* s, void* grad, double* loss,
                     ic_loss_terms* terms);

/* Vector-Jacobian product s_bar = J^T delta_bar of s -> delta_s (no prior);
 * all device buffers of n_part^3.  Returns IC_ERR_NONFINITE when s is not
 * finite. */
int ic_vjp(ic_ctx* ctx, const void* s, const void* delta_bar, void* s_bar);

/* In-place rank-order matching and projection of the white noise s
 * (sections 2.3.1-2.3.2), in the order real-space matching on M = 1 cells,
 * Fourier-space matching per k bin (of |z| to Rayleigh draws, phases kept,
 * with IC_ROM_FOURIER; of Re z and Im z together to N(0, 1/2) draws with
 * IC_ROM_FOURIER_REIM), projection P (z-score and reset of |s| > s_th,
 * repeated until a pass resets nothing, so the result has mean 0, std 1
 * and no extremes); flags selects the parts.  event keys the random draws
 * (reset draws also use trial).  info is optional; its n_fourier counts
 * matched modes under either reading.  A rank-order pass fails with
 * IC_ERR_NONFINITE on NaN; both Fourier flags together give
 * IC_ERR_INVALID_ARG. */
int ic_project_rankmatch(ic_ctx* ctx, void* s, uint32_t flags, uint64_t event,
                         int32_t trial, ic_rom_info* info);

/* One projected L-BFGS iteration (section 2.3.1): direction from the
 * two-loop recursion over the stored pairs (FP64 dot products) with initial
 * inverse Hessian gamma I, gamma = S.Y / Y.Y of the newest pair, or 1/|g|
 * with an empty history (the first step of a fresh history, -g/|g|, has unit
 * length), backtracking
 * line search along the projection arc s' = P(s + eps p) from eps_max,
 * halving, accepting when g.(s' - s) < 0, L(s') < L and
 * L(s') <= L + c1 g.(s' - s);
 * if that fails for a quasi-Newton direction, the history is reset and
 * steepest descent is searched once more.  Then the (S, Y) pair update.
 * s, grad: device in/out (n_part^3); loss: host in/out; iteration keys the
 * reset draws.  Returns IC_ERR_LINESEARCH when no trial passes or the
 * gradient is zero (s, grad and loss are then unchanged), IC_ERR_NONFINITE
 * when s, the loss or the gradient is not finite. */
int ic_lbfgs_step(ic_ctx* ctx, void* s, void* grad, double* loss, int64_t iteration,
                  ic_lbfgs_info* info);

/* Clears the L-BFGS history (after a rank-order matching event). */
int ic_lbfgs_reset(ic_ctx* ctx);

/* White-noise upsampling between the levels of the resolution schedule
 * (section 3: the run at the coarse resolution seeds the full-resolution
 * one).  The paper does not say how the noise moves to the finer grid; the
 * reading here keeps the large-scale modes and draws fresh small-scale ones.
 * s_high (device, n_part^3 of high) = inverse DFT of Z, where Z is the DFT of
 * fresh N(0,1) noise (Philox stream 4, counter (j, 0, 4, event), j the
 * lattice index) except on the modes whose three wave indices all lie
 * strictly inside (-n_low/2, n_low/2), which hold the DFT of s_low (device,
 * n_low^3 of low) times (n_part / n_low)^{3/2}; the coarse Nyquist modes are
 * not carried.  The DFT is unnormalised, so unit-variance white noise stays
 * unit-variance.  low must have the same precision and box and half the
 * particle grid side of high.  Runs on high's stream (low's transform too;
 * low's stream is restored).  Uses high's spectrum workspace; s_low is read
 * only.  Errors (reported on high): IC_ERR_INVALID_ARG for a null or
 * mismatched context or a null field. */
int ic_upsample_noise(ic_ctx* high, ic_ctx* low, const void* s_low, void* s_high,
                      uint64_t event);

#ifdef __cplusplus
}
#endif

#endif /* IC_API_H */
