/*
 * histfit.h -- C ABI of the MI355X (gfx950) histogram-fit library.
 *
 * The library evaluates a binned fit objective and its reverse-mode gradient
 * with respect to the model parameters, and fits histograms with it.  This is
 * the computation the paper accelerates with AD (sec. 4 "Integration and
 * Results", Fig. 2a: a parametric function fitted to a uniformly binned
 * histogram with an AD-generated gradient; sec. 2 "Background": reverse
 * accumulation gives the gradient of a scalar objective at a cost independent
 * of the number of parameters).  The gradient routine takes the inputs and
 * caller-provided output adjoints for the selected parameters, as the
 * generated gradient of Listing 1 (sec. 3) does.
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.   Every array argument is a DEVICE pointer on the context's GPU
 *           unless stated otherwise.  The caller owns all inputs and outputs;
 *           the library never frees caller memory.  Descriptor structs
 *           (hf_hist, hf_model, hf_fit_opts) are read on the host during the
 *           call and may be reused at once.
 * Streams.  Work is enqueued on `stream` (a hipStream_t; NULL is the null
 *           stream) and is asynchronous: outputs are valid once the stream has
 *           been synchronised.  No call synchronises the stream.
 * Returns.  0 on success or a negative hf_error code for what the host can
 *           check (null pointers, sizes, dtypes, unsupported combinations,
 *           HIP launch errors).  hf_last_error() gives the message.
 * Status.   Data-dependent conditions never fail the call; they are written
 *           to a device status word (bit field, hf_bin_status) so that no
 *           call forces a host synchronisation:
 *             HF_ST_DOMAIN     a bin had mu <= 0 where the objective needs
 *                              mu > 0; the NLL is +inf and, the objective
 *                              not being differentiable there, the gradient
 *                              is NaN;
 *             HF_ST_NONFINITE  theta held a NaN or infinity; the NLL and
 *                              gradient outputs are then NaN.
 * Threads.  A context is not thread safe and its calls must not overlap:
 *           use one context per host thread or per concurrently used stream.
 *           Calls serialised on one stream may share a context.
 * Results.  Reductions run in a fixed order: repeated calls with the same
 *           inputs on the same GPU give bit-identical outputs.
 *
 * Models (theta layout, all FP64)
 * -------------------------------
 *   HF_GAUSS_POLY  1D: sum over n_gauss Gaussians A exp(-((x-m)/s)^2/2),
 *                  theta = (A,m,s) per Gaussian, then the polynomial
 *                  background sum_{j=0..poly_degree} c_j t^j with
 *                  t = (x - t_shift)/t_scale; poly_degree = -1: no background.
 *                  The amplitude form matches the "gaus" function
 *                  {Constant, Mean, Sigma} that Fig. 2a fits.
 *   HF_GAUSS_EXP   1D: the same Gaussians plus exp(b0 + b1 t), theta ends
 *                  with (b0, b1).
 *   HF_GAUSS2D     2D: A exp(-Q/2) + c, Q = (u^2 - 2 rho u v + v^2)/(1-rho^2),
 *                  u = (x-mx)/sx, v = (y-my)/sy;
 *                  theta = (A, mx, my, sx, sy, rho, c).
 * Supported sizes: 0 <= n_gauss <= 4 and -1 <= poly_degree <= 3 (at least
 * one term), so P = hf_model_nparams() <= 16.
 * The model is evaluated at bin centres x_i = lo + (i + 1/2)(hi - lo)/n.
 *
 * Objectives (per bin, count n, model mu, optional weight w; L = sum w l)
 * -----------------------------------------------------------------------
 *   HF_NEYMAN   l = (n - mu)^2 / n, bins with n = 0 skipped.
 *   HF_PEARSON  l = (n - mu)^2 / mu.
 *   HF_POISSON  l = mu - n + n ln(n/mu) (n > 0),  l = mu (n = 0): the
 *               Poisson negative log-likelihood minus its saturated value
 *               (no factor 2); same minimiser and gradient as
 *               sum(mu - n ln mu).
 *
 * Precision
 * ---------
 *   HF_FP64      every per-bin step in FP64.
 *   HF_FP32_BIN  the per-bin transcendental and reciprocal steps use FP32
 *                hardware instructions (bin centres and x - m stay FP64);
 *                NLL and gradient are accumulated in FP64 either way.
 */
#ifndef HISTFIT_H
#define HISTFIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hf_stream_t; /* same type as hipStream_t */
typedef struct hf_ctx hf_ctx;

typedef enum {
  HF_OK = 0,
  HF_EINVAL = -1,       /* null pointer, bad size, dtype or parameter count */
  HF_EUNSUPPORTED = -2, /* model/objective/precision combination not built */
  HF_EHIP = -3,         /* a HIP runtime call failed                        */
  HF_ENOMEM = -4,       /* device scratch could not be allocated            */
  HF_ECAPTURE = -5      /* scratch would have to grow during stream capture */
} hf_error;

typedef enum { HF_NEYMAN = 0, HF_PEARSON = 1, HF_POISSON = 2 } hf_objective;
typedef enum { HF_GAUSS_POLY = 1, HF_GAUSS_EXP = 2, HF_GAUSS2D = 3 } hf_model_kind;
typedef enum { HF_FP64 = 0, HF_FP32_BIN = 1 } hf_precision;
typedef enum { HF_U32 = 0, HF_F32 = 1, HF_F64 = 2 } hf_dtype;
typedef enum { HF_ST_DOMAIN = 1, HF_ST_NONFINITE = 2 } hf_bin_status;

typedef struct {
  int32_t kind;        /* hf_model_kind                                   */
  int32_t n_gauss;     /* 0..4 (HF_GAUSS2D: ignored)                      */
  int32_t poly_degree; /* -1..3 (HF_GAUSS_POLY only)                      */
  int32_t bin_average; /* 0: mu_i is the model at the centre of bin i;
                          1: its average over bin i (integral / width):
                          erf differences per Gaussian, exact averages of
                          t^j and of exp(b0 + b1 t); 1D models with
                          nll_eval / nll_grad in HF_FP64 only,
                          HF_EUNSUPPORTED elsewhere                       */
  double t_shift;      /* background variable t = (x - t_shift)/t_scale   */
  double t_scale;      /* nonzero                                         */
} hf_model;

typedef struct {
  const void* counts;   /* device, nx*ny values of counts_dtype, row-major
                           with x fastest; 16-byte aligned                 */
  const float* weights; /* device f32[nx*ny] per-bin weights, or NULL (1);
                           16-byte aligned                                 */
  int64_t nx;           /* bins along x, >= 1                              */
  int64_t ny;           /* bins along y; 1 for the 1D models               */
  int32_t counts_dtype; /* hf_dtype                                        */
  int32_t reserved;     /* must be 0                                       */
  double xlo, xhi;      /* x range, xhi > xlo (ignored with x_edges)       */
  double ylo, yhi;      /* y range (2D only), yhi > ylo                    */
  const double* x_edges; /* NULL: nx uniform bins on [xlo, xhi].  Else
                           device f64[nx + 1], ascending: 1D bins of any
                           widths, bin i spanning [x_edges[i],
                           x_edges[i+1]]; the model is taken at the bin's
                           midpoint, or averaged over it (bin_average).
                           nll_eval / nll_grad in HF_FP64 only; edges that
                           are not ascending give undefined values (never
                           an out-of-bounds access).                      */
} hf_hist;

/* Creates a context on HIP device `device` and makes it current for the
 * calling thread.  The context owns the device scratch used by reductions
 * and fits (per-block partial sums, a completion ticket, the log table, the
 * fit work queue and the 65,536-entry longest-first ordering buffer).  All
 * of it is allocated here, once, and freed only by hf_ctx_destroy: no other
 * call allocates, frees or synchronises, so every call may be captured into
 * a HIP graph, and a graph captured earlier stays valid after later calls
 * of any size.  HF_ECAPTURE is reserved; no call returns it.              */
int hf_ctx_create(hf_ctx** out, int device);
void hf_ctx_destroy(hf_ctx* ctx);
/* Message of the last failing call on ctx (empty string if none); valid
 * until the next call on ctx.  With ctx NULL: the message of the calling
 * thread's last failing context-free call (nll_grad_noalloc), or "".      */
const char* hf_last_error(const hf_ctx* ctx);

/* Number of parameters P of a model, or HF_EINVAL / HF_EUNSUPPORTED.      */
int hf_model_nparams(const hf_model* model);

/* NLL value: the fit objective L(theta) = sum_i w_i l(n_i, mu_i(theta))
 * over every bin, the function whose parameter gradient the paper's
 * histogram-fitting application differentiates (sec. 4, Fig. 2a: a TH1D
 * fitted with a TF1 of Gaussians).
 *   theta      device f64[P], read on the device (no host copy).
 *   nll_out    device f64[1], overwritten with L(theta).
 *   status_out device i32[1] or NULL, overwritten with the hf_bin_status
 *              bits of this evaluation.                                   */
int nll_eval(hf_ctx* ctx, const hf_hist* hist, const hf_model* model, int32_t objective,
             int32_t precision, const double* theta, double* nll_out, int32_t* status_out,
             hf_stream_t stream);

/* NLL and its reverse-mode gradient, in one pass over the bins: the
 * adjoint of L propagated back through every bin's model evaluation to the
 * parameters (sec. 2: reverse accumulation costs a small multiple of one
 * function evaluation whatever P is; sec. 3: reads of theta shared by all
 * bins become adjoint writes by all bins, summed here in a fixed order;
 * Listing 1: the caller supplies the storage the adjoints are written to).
 *   seed       device f64[1] upstream adjoint dOut/dL, or NULL for 1.
 *   nll_out    device f64[1], overwritten with L(theta) (not scaled by seed).
 *   grad_out   device f64[P], OVERWRITTEN (not accumulated) with
 *              seed * dL/dtheta; entries whose bit is clear in free_mask are
 *              set to 0.  free_mask = 0 selects every parameter.
 *   grad_w_out device f32[nx*ny] or NULL, 16-byte aligned: seed * dL/dw_i =
 *              seed * l_i per bin (unspecified for domain-error bins).
 *   status_out as for nll_eval.                                           */
int nll_grad(hf_ctx* ctx, const hf_hist* hist, const hf_model* model, int32_t objective,
             int32_t precision, const double* theta, const double* seed, double* nll_out,
             double* grad_out, float* grad_w_out, uint32_t free_mask, int32_t* status_out,
             hf_stream_t stream);

/* nll_grad without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same computation and outputs as nll_grad, with the
 * reduction scratch in a file-scope device array of the library (296 KiB
 * per GPU, held until the process ends: the block partials of up to 2048
 * blocks x 17 values, their status flags and the log table).  No call
 * allocates or frees device memory; the first call on a device (with that
 * device current) looks up the array's address there and copies the log
 * table into it.  The kernels run on the calling thread's current device.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or threads) race and give wrong results; calls
 * serialised on one stream do not.  Each call overwrites every partial it
 * reads, so nothing needs clearing between calls.  Returns HF_EINVAL for a
 * model of more than 16 parameters (the partials the array holds per
 * block), and the errors of nll_grad otherwise; hf_last_error(NULL) gives
 * the message of this thread's last failing call.                          */
int nll_grad_noalloc(const hf_hist* hist, const hf_model* model, int32_t objective,
                     int32_t precision, const double* theta, const double* seed, double* nll_out,
                     double* grad_out, float* grad_w_out, uint32_t free_mask,
                     int32_t* status_out, hf_stream_t stream);

/* Extended unbinned NLL and its reverse-mode gradient: the binned
 * objective's per-bin evaluation applied to single events at arbitrary
 * positions (the per-event batch evaluation of RooFit-style likelihoods the
 * paper's outlook names, sec. 5).  A 1D model is read as an
 * intensity lambda(x; theta) (events per unit x):
 *   L(theta) = Lambda(theta) - sum_e w_e ln lambda(x_e),
 *   Lambda   = integral of lambda over [lo, hi] (closed form through erf),
 * the Poisson-process likelihood, i.e. the binned Poisson objective in the
 * limit of single-event bins.
 *   events     device f64[n_events], 16-byte aligned for the vector path
 *              (any alignment works); events outside [lo, hi] are skipped.
 *   weights    device f32[n_events] or NULL (1).
 *   theta      device f64[P];  nll_out device f64[1], overwritten.
 *   grad_out   device f64[P], OVERWRITTEN with dL/dtheta, or NULL for the
 *              value alone.
 *   status_out device i32[1] or NULL: HF_ST_DOMAIN when lambda <= 0 at an
 *              event inside the range (L = +inf, gradient NaN),
 *              HF_ST_NONFINITE when theta is not finite (outputs NaN).
 * 1D models only (HF_EUNSUPPORTED for HF_GAUSS2D).  Uses the
 * context's reduction scratch: calls on one context must not overlap.     */
int nll_unbinned(hf_ctx* ctx, const double* events, const float* weights, int64_t n_events,
                 double lo, double hi, const hf_model* model, const double* theta,
                 double* nll_out, double* grad_out, int32_t* status_out, hf_stream_t stream);

/* Expected Hessian (Fisher information) of the objective at theta: the
 * second-derivative matrix that the paper (sec. 4) leaves to numerical
 * differentiation, in the Gauss-Newton form that parameter errors use,
 *   F_jk = sum_i w_i c_i (dmu_i/dtheta_j)(dmu_i/dtheta_k),
 *   c_i = 1/mu_i (Poisson), 2/mu_i (Pearson), 2/n_i (Neyman, n_i > 0);
 * bins whose c_i is not finite and positive are skipped.  Only the Neyman
 * objective reads the counts.  FP64 throughout.
 *   theta      device f64[P].
 *   fisher_out device f64[P*P], row-major, OVERWRITTEN (symmetric); all NaN
 *              when theta is not finite.
 *   status_out device i32[1] or NULL: HF_ST_NONFINITE when theta is not
 *              finite, else 0.
 * Uses the context's reduction scratch, like nll_grad: calls on one context
 * must not overlap in time.                                               */
int hf_nll_fisher(hf_ctx* ctx, const hf_hist* hist, const hf_model* model, int32_t objective,
                  const double* theta, double* fisher_out, int32_t* status_out,
                  hf_stream_t stream);

/* Parameter covariance from B Fisher matrices (hf_nll_fisher's layout):
 * for the free parameters (free_mask bit set; 0 = all),
 *   cov = 2 UP F^-1,  UP = 1/2 (Poisson NLL, which has no factor 2) or 1
 *   (chi-square): the inverse curvature at the level where the objective
 *   rises by UP, so sqrt(cov_kk) is the usual one-sigma error;
 * rows and columns of fixed parameters are 0.  The inverse is taken by
 * Cholesky of F scaled to unit diagonal; a pivot not above 1e-12 (or a
 * non-positive diagonal entry) makes the free entries NaN and status 1.
 *   fisher     device f64[B][P][P];  cov_out device f64[B][P][P];
 *   status_out device i32[B] or NULL (0 ok, 1 not positive definite).
 *   P          1..16.                                                      */
int hf_fisher_covariance(hf_ctx* ctx, int32_t B, int32_t P, int32_t objective,
                         const double* fisher, uint32_t free_mask, double* cov_out,
                         int32_t* status_out, hf_stream_t stream);

/* Elementwise Gaussian and its reverse-mode gradient over n independent
 * parameter sets: the device-function example of paper sec. 3 (Listing 1),
 * one element per thread, generalised to shared parameters.  Per element,
 * with d = x_i - p_i and s = sigma_i,
 *   g_i = (2 pi)^(-1/2) s^(-a) exp(-d^2 / (2 s^2)),
 *   a = 1/2 (HF_NORM_LISTING: the normalisation as the listing prints it)
 *       or 1 (HF_NORM_PDF: the normal probability density);
 * with upstream adjoint w_i (seed_i, or 1 when seed is NULL):
 *   dx_i = w_i dg_i/dx_i = -w_i g_i d / s^2,  dp_i = -dx_i,
 *   dsigma_i = w_i g_i (d^2 / s^3 - a / s).
 * p (resp. sigma) is either per element (p_shared = 0: p is f64[n]) or one
 * value for all elements (p_shared = 1: p is f64[1]).  A shared input's
 * adjoint is the sum over the elements, dp_out[0] = sum_i dp_i, taken in a
 * fixed order (deterministic); a per-element input's adjoint is per element.
 *   x          device f64[n];  seed device f64[n] or NULL.
 *   g_out, dx_out              device f64[n] or NULL (not computed).
 *   dp_out, dsigma_out         device f64[n] (per element), f64[1] (shared),
 *                              or NULL.  All outputs are OVERWRITTEN.
 *   sigma must be positive for HF_NORM_LISTING (s^(-1/2)) and nonzero for
 *   HF_NORM_PDF; other values follow IEEE arithmetic (NaN or inf).
 * n may be 0 (shared adjoints are then 0).  Arrays that are all 16-byte
 * aligned move as 16-byte vectors.  A call with a shared input uses the
 * context's reduction scratch: calls on one context must not overlap.     */
typedef enum { HF_NORM_LISTING = 0, HF_NORM_PDF = 1 } hf_gauss_norm;
int hf_gauss_grad_map(hf_ctx* ctx, int64_t n, const double* x, const double* p, int32_t p_shared,
                      const double* sigma, int32_t sigma_shared, int32_t norm, const double* seed,
                      double* g_out, double* dx_out, double* dp_out, double* dsigma_out,
                      hf_stream_t stream);

/* Options of the fitter: BFGS on the inverse Hessian in scaled coordinates,
 * backtracking Armijo line search (c1 = 1e-4, step halved up to ls_max
 * times), stop when EDM = g^T H g / 2 < max(edm_tol, 4 eps |L|).  The
 * first inverse Hessian is the identity, or with hessian_init = 1 the
 * inverse of the expected Hessian (Fisher information) at theta0,
 *   F = sum_i c_i (dmu_i/dtheta)(dmu_i/dtheta)^T,
 *   c_i = d^2 l/d mu^2 at n_i = mu_i (1/mu Poisson, 2/mu Pearson, 2/n for
 *   n > 0 Neyman), bins whose c_i is not finite and positive skipped,
 * taken by Cholesky in the scaled coordinates; it falls back to the
 * identity when a pivot is not above 1e-12 times the largest diagonal
 * entry or a value is not finite.  The first step is then a Fisher-scoring
 * (Gauss-Newton) step, and no first-update scaling is applied.            */
typedef struct {
  int32_t max_iter;     /* iteration limit, >= 1                          */
  int32_t ls_max;       /* line-search halvings, 1..60                    */
  int32_t fixed_iters;  /* nonzero: ignore the EDM test (timing runs)     */
  uint32_t free_mask;   /* bit k set: theta_k is fitted; 0 = all          */
  double edm_tol;       /* convergence threshold on EDM                   */
  double polish_edm;    /* HF_FP32_BIN: switch to FP64 bins once EDM is
                           below this (<= 0: never switch)                */
  int32_t hessian_init; /* 0: identity; 1: inverse expected Hessian       */
  int32_t gradient;     /* 0: reverse-mode adjoint sweep (value and
                           gradient in one pass); 1: central differences
                           of the value, g_q = (L(u + h e_q) - L(u - h e_q))
                           / 2h in the scaled coordinates, h = 1e-4
                           max(1, |u_q|): 2 nf value sweeps per gradient,
                           taken only at accepted points (the line search
                           needs values only).  1 requires HF_FP64.      */
} hf_fit_opts;

/* Per-fit status codes written to status[b] by fit_batch.                */
typedef enum {
  HF_FIT_CONVERGED = 0,
  HF_FIT_MAXITER = 1,
  HF_FIT_LSFAIL = 2,
  HF_FIT_NONFINITE = 3,
  HF_FIT_DOMAIN = 4,
  HF_FIT_BADHIST = 5 /* offsets[b+1] <= offsets[b] or a bad range        */
} hf_fit_status;

/* Fits B independent 1D histograms in one launch: the paper's histogram
 * fit (sec. 4, Fig. 2a and 2b: a gradient-driven minimisation of the fit
 * objective, the gradient taken by reverse mode or, for comparison, by
 * central differences) repeated over a batch, one persistent workgroup per
 * fit at a time.  Batches of up to 65,536 histograms are taken longest
 * first; larger batches in index order.
 *   counts_concat device array of counts_dtype: histogram b occupies
 *                 [offsets[b], offsets[b+1]).
 *   offsets       device i64[B+1], offsets[0] = 0, nondecreasing.
 *   ranges        device f64[2B]: (lo_b, hi_b).
 *   theta0        device f64[B*P] start points; theta_out device f64[B*P]
 *                 canonicalised results (|s|, Gaussians ordered by mean).
 *   nll_out       device f64[B]: final L, re-evaluated with FP64 bins.
 *   status, iters, nevals  device i32[B]: hf_fit_status, BFGS iterations,
 *                 objective evaluations.
 * Only HF_GAUSS_POLY and HF_GAUSS_EXP models.                             */
int fit_batch(hf_ctx* ctx, int32_t B, const void* counts_concat, int32_t counts_dtype,
              const int64_t* offsets, const double* ranges, const hf_model* model,
              int32_t objective, int32_t precision, const double* theta0, const hf_fit_opts* opts,
              double* theta_out, double* nll_out, int32_t* status, int32_t* iters,
              int32_t* nevals, hf_stream_t stream);


/* Launch shape of fit_batch on this context (the autotuner's knobs):
 * wg_per_cu persistent workgroups per compute unit (1..16, default 2);
 * cache_bins: histograms of u32 counts with at most this many bins are copied
 * once into LDS and every evaluation reads them there (0 = never; at most
 * hf_fit_max_cache_bins() for the block size, checked by fit_batch);
 * block_size: threads per workgroup, each fit's bins shared among them (256
 * = one wave per SIMD, default; or 512).  The results do not depend on the
 * shape beyond summation order.  Host-only calls; HF_EINVAL for values out
 * of range.                                                               */
int hf_fit_set_tuning(hf_ctx* ctx, int32_t wg_per_cu, int32_t cache_bins, int32_t block_size);
int hf_fit_get_tuning(const hf_ctx* ctx, int32_t* wg_per_cu, int32_t* cache_bins,
                      int32_t* block_size);
/* One wave per small histogram in fit_batch (a schedule knob like those
 * of hf_fit_set_tuning): once the longest-first queue reaches histograms of
 * at most wave_bins bins, every wave of a workgroup fits its own histogram,
 * its state and (u32 counts) an LDS copy of the counts in a slot of its
 * own, with wave-level reductions and no workgroup barriers; larger
 * histograms keep a whole workgroup each.  0 (default) turns it off; it also
 * stays off for batches above 65,536 histograms, which run unsorted.  At
 * most hf_fit_max_wave_bins() for the model, objective and block size,
 * checked by fit_batch (HF_EINVAL).  The results do not depend on it beyond
 * summation order.  Host-only; HF_EINVAL for wave_bins < 0.
 * hf_fit_get_wave_bins returns the setting (or HF_EINVAL for NULL).      */
int hf_fit_set_wave_bins(hf_ctx* ctx, int32_t wave_bins);
int hf_fit_get_wave_bins(const hf_ctx* ctx);
int hf_fit_max_wave_bins(hf_ctx* ctx, const hf_model* model, int32_t objective,
                         int32_t block_size);

/* Largest cache_bins the fit kernel of this model and objective, with
 * workgroups of block_size threads, can hold in LDS next to its own state
 * (>= 0), or a negative hf_error.                                         */
int hf_fit_max_cache_bins(hf_ctx* ctx, const hf_model* model, int32_t objective,
                          int32_t block_size);

/* ------------------------------------------------------------------------
 * Learned initialiser: a dense GELU network 256 -> 512 -> 512 -> 512 -> 5
 * that predicts fit starting parameters of the Gauss + exponential model
 * from a 256-bin rebinned, log-normalised histogram.  It is trained on the
 * results of plain fits (fit_batch from hf_default_starts) and used as the
 * start of the same fitter, with the plain start as fallback.  Dense layers
 * run on BF16 MFMA with FP32 accumulation; master weights, Adam moments and
 * the loss are FP32.
 *
 * Flat FP32 parameter layout (offsets in floats, row-major [out][in]):
 *   W1[512][256] b1[512] W2[512][512] b2[512] W3[512][512] b3[512]
 *   W4[32][512] b4[32]; rows 5..31 of W4 and b4[5..31] are padding and must
 *   be zero (they then stay zero).  Total hf_mlp_nparams() floats.
 * Target space (per fit, 5 values): (m, ln|s|, ln A, b0, b1), standardised by
 * per-column mean and standard deviation.
 * Batch sizes must be multiples of 64.  Every call returns HF_EINVAL (and
 * launches nothing) for a batch that is not, a NULL pointer argument, or a
 * workspace smaller than hf_mlp_workspace_bytes(batch); shapes of the other
 * buffers cannot be checked through plain pointers and are the caller's.
 * ---------------------------------------------------------------------- */
enum { HF_MLP_IN = 256, HF_MLP_HIDDEN = 512, HF_MLP_OUT = 5, HF_MLP_OUT_PAD = 32 };

int64_t hf_mlp_nparams(void);
/* Device scratch a forward or training step of `batch` rows needs (bytes);
 * HF_EINVAL (negative) for a batch that is not a positive multiple of 64.  */
int64_t hf_mlp_workspace_bytes(int32_t batch);
/* Where a workspace of `batch` rows keeps the network's stored values, as
 * byte offsets from its start (for inspecting them after a call, e.g. to
 * check each layer against a reference element by element).  offsets
 * (host int64[12]) receives, in order:
 *   a0 a1 a2 a3   BF16 [batch][in_l] layer inputs: a0 = bf16(x), a_l the
 *                 rounded GELU outputs of hidden layer l;
 *   z1 z2 z3      FP32 [batch][512] hidden pre-activations (training step
 *                 only);
 *   y             FP32 [batch][32] network output (training step only);
 *   dz1 .. dz4    BF16 [batch][out_l] adjoints of the pre-activations of
 *                 layers 1..4 (training step only).
 * Returns 0, or HF_EINVAL for a batch that is not a positive multiple of 64
 * or a NULL offsets.  Host-only.                                          */
int hf_mlp_workspace_layout(int32_t batch, int64_t* offsets);

/* Rebins histogram b of counts_concat (offsets as in fit_batch) to 256 coarse
 * bins -- fine bin i goes to coarse bin floor((i + 1/2) 256 / nbins) -- and
 * writes out[b][j] = (log1p(c_j / k_j) - in_mean) / in_std, with c_j the
 * summed counts and k_j the number of fine bins of coarse bin j (0 if none).
 * out: device f32[B][256].                                                */
int hf_rebin_lognorm(hf_ctx* ctx, int32_t B, const void* counts_concat, int32_t counts_dtype,
                     const int64_t* offsets, float in_mean, float in_std, float* out,
                     hf_stream_t stream);

/* The plain method's starting point for one Gaussian + exp(b0 + b1 t)
 * (model: HF_GAUSS_EXP, n_gauss = 1), per histogram of a batch laid out as
 * in fit_batch:
 *   background: mean counts bk0, bk1 of the first and last 4% of the bins
 *     (at least one bin, floored at 1), an exponential through the two
 *     block centres c0, c1: bg_i = exp(ln bk0 + (ln bk1 - ln bk0)
 *     (i + 1/2 - c0)/(c1 - c0)) in counts per bin;
 *   peak: the largest integer excess E_i = rint(S_i - (2W+1) bg_i), S_i the
 *     sum of the counts of bins i-W..i+W, W = max(1, nbins/256), over
 *     W <= i < nbins - W, lowest index on ties; A = max(E/(2W+1), 1);
 *   width: the excess walked outwards from the peak until 2 E < E_max gives
 *     the FWHM; s = FWHM/2.3548 clamped to [0.005, 0.1] of the range.
 * theta0: device f64[B][5] (A, m, s, b0, b1).                              */
int hf_default_starts(hf_ctx* ctx, int32_t B, const void* counts_concat, int32_t counts_dtype,
                      const int64_t* offsets, const double* ranges, const hf_model* model,
                      double* theta0, hf_stream_t stream);

/* Per-column mean and population standard deviation of x[n][cols] (device
 * f32), summed in FP64 in a fixed order; mean, std: device f32[cols].       */
int hf_column_stats(hf_ctx* ctx, int64_t n, int32_t cols, const float* x, float* mean, float* std,
                    hf_stream_t stream);

/* theta (device f64[B][5], Gauss + exp model) -> standardised targets
 * (device f32[B][5]): ((m, ln|s|, ln A, b0, b1) - mean)/std.  With mean = 0
 * and std = 1 it gives the raw target values (for hf_column_stats).      */
int hf_theta_to_target(hf_ctx* ctx, int32_t B, const double* theta, const float* mean,
                       const float* std, float* target, hf_stream_t stream);
/* Network outputs (device f32[B][32], first 5 columns) -> theta (f64[B][5]). */
int hf_target_to_theta(hf_ctx* ctx, int32_t B, const float* y, const float* mean,
                       const float* std, double* theta, hf_stream_t stream);

/* Forward pass: y = network(x).  params: device f32[hf_mlp_nparams()];
 * x: device f32[batch][256]; y: device f32[batch][32] (columns 5..31 are the
 * padding outputs); workspace: device scratch of workspace_bytes >=
 * hf_mlp_workspace_bytes(batch) bytes, 256-byte aligned, owned by the caller
 * and not to be used by another call until this one has completed on
 * `stream`.                                                                */
int hf_mlp_forward(hf_ctx* ctx, int32_t batch, const float* params, const float* x, float* y,
                   void* workspace, int64_t workspace_bytes, hf_stream_t stream);

/* One AdamW step (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay
 * wd) on the mean squared error over the 5 target columns:
 * loss = sum (y - target)^2 / (5 batch).  params, adam_m, adam_v: device
 * f32[hf_mlp_nparams()], updated in place; step: 1-based step count (bias
 * correction); grads: device f32[hf_mlp_nparams()] receives the gradient of
 * this step; loss_out: device f32[1].  Rounding points: x, weights,
 * activations and output/hidden adjoints are rounded to BF16 (nearest even)
 * before each product; products accumulate in FP32.  target: device
 * f32[batch][5]; workspace as for hf_mlp_forward.  HF_EINVAL also for
 * step < 1, lr <= 0 or wd < 0.                                             */
int hf_mlp_train_step(hf_ctx* ctx, int32_t batch, float* params, float* adam_m, float* adam_v,
                      int32_t step, float lr, float wd, const float* x, const float* target,
                      float* grads, float* loss_out, void* workspace, int64_t workspace_bytes,
                      hf_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HISTFIT_H */
