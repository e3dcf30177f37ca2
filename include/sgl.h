/*
 * sgl.h -- fast SGL Fourier transform for scattered data (NFSGLFT) and its
 * adjoint on AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Wuelker, "Fast SGL Fourier transforms for scattered
 * data", Def. 1.3 and eq. (1.2)): for M points x_i in R^3 and bandwidth B,
 *     f = Lambda fhat,   Lambda[i, mu] = H_{n(mu) l(mu) m(mu)}(x_i),
 * with the SGL basis functions H_nlm of Def. 1.1 and the coefficient order
 * mu = n(n-1)(2n-1)/6 + l(l+1) + m (Section 1).  The adjoint is Lambda^H
 * (Section 1, the paragraph after eq. (1.3)).  Both are computed by the fast
 * algorithm of Section 6 (Thm. 6.2, Cor. 6.3): a radial and a polar
 * conversion into the coefficients eta of a 3D trigonometric polynomial
 * (eq. nfsglft_nfft) on the 4B x 2B x 2B grid of Remark 8.1, followed by the
 * Gaussian-window NFFT of Section 2 on the oversampled grid sigma*n.  Only
 * the NFFT is approximate (Section 7); its error falls at least
 * exponentially in the cutoff q (Thm. 2.7).
 *
 * Conventions shared by every entry point
 *  - Memory: all data pointers are DEVICE pointers owned by the caller; the
 *    library never frees them.  A plan owns its tables and workspace.
 *  - Complex data are interleaved (re, im): double2 for SGL_F64, float2 for
 *    SGL_F32 (the layout of torch.complex128 / torch.complex64).
 *  - Points are Cartesian (x, y, z) rows, M x 3, double for SGL_F64 and
 *    float for SGL_F32.  The point transform itself always runs in FP64.
 *  - Streams: every call enqueues on the plan's stream and returns without a
 *    host synchronisation, except sgl_plan, which is synchronous.
 *  - Errors: status codes only, nothing is thrown across the ABI.  Argument
 *    checks run on the host before any work is enqueued; on error, outputs
 *    are unspecified and nothing has been written to them.  Inputs and
 *    outputs must not overlap (SGL_E_INVAL).  A plan must not be used from
 *    two host threads at once.
 */
#ifndef SGL_H
#define SGL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgl_plan_s *sgl_plan_t;

typedef enum {
  SGL_OK = 0,
  SGL_E_INVAL = -1,       /* bad argument, null pointer, aliasing, non-finite point */
  SGL_E_RANGE = -2,       /* user rho smaller than max_i |x_i|                      */
  SGL_E_NOMEM = -3,       /* device or host allocation failed                       */
  SGL_E_DEVICE = -4,      /* HIP runtime or launch error                            */
  SGL_E_UNSUPPORTED = -5  /* e.g. a bandwidth whose FFT grid exceeds 2048 x 1024^2  */
} sgl_status;

typedef enum { SGL_F64 = 0, SGL_F32 = 1 } sgl_precision;

/* Replace the NFFT by the exact NDFT of Def. 2.4 (the variant the paper uses
 * to separate the NFFT error from the rest, Section 8, fourth test).  O(B^3)
 * work per point: for testing only. */
#define SGL_FLAG_EXACT_NDFT (1u << 0)
/* Conversion products (Thm. 6.2, Cor. 6.3) on the FP16 matrix cores with hi/lo
 * split operands and FP32 accumulation (tables built in long double and split
 * at plan time, per row; data split per column).  Keeps about 22 bits of every
 * product; the conversion sums cancel strongly when the radial functions grow
 * towards rho, so results are less accurate than the default FP64 products
 * (errors per workload are stated with the design notes).  Bandwidths above
 * SGL_CONV_SPLIT16_MAX_B are refused (SGL_E_UNSUPPORTED, a host-side check):
 * at B = 64 the adjoint misses 1e-5 relative to the direct sum. */
#define SGL_FLAG_CONV_SPLIT16 (1u << 1)
#define SGL_CONV_SPLIT16_MAX_B 48

typedef struct {
  int32_t B;          /* bandwidth, 2 <= B <= 256 (Section 6 assumes B >= 2)              */
  int32_t sigma;      /* integer oversampling factor, 2..4 (Section 2; Thm. 2.7 needs >= 2) */
  int32_t q;          /* window cutoff, 1 <= q and 2q <= sigma*2B (q < sigma n, Section 2)  */
  double rho;         /* <= 0: rho = max_i |x_i| (eq. nfsglft_rho); else >= max_i |x_i|     */
  int32_t precision;  /* sgl_precision                                                      */
  uint32_t flags;     /* SGL_FLAG_*                                                         */
} sgl_params;

/* Number of coefficients B(B+1)(2B+1)/6 (Section 1); -1 if B < 1. */
int64_t sgl_num_coeffs(int32_t B);

/* mu(n,l,m) = n(n-1)(2n-1)/6 + l(l+1) + m for |m| <= l < n (Section 1); -1 otherwise. */
int64_t sgl_coeff_index(int32_t n, int32_t l, int32_t m);

/* Reduced trigonometric grid of Remark 8.1: dims[0..2] = {4B, 2B, 2B}.
 * eta buffers used by the stage entry points are dims[0]*dims[1]*dims[2]
 * complex values, index ((k0 + 2B) * 2B + (k1 + B)) * 2B + (k2 + B) for
 * k0 in [-2B, 2B), k1, k2 in [-B, B) -- the index sets I_{4B} x I_{2B} x I_{2B}. */
sgl_status sgl_eta_dims(int32_t B, int32_t dims[3]);

/* Create a plan for M points (Section 6 setup): validates the parameters,
 * computes the transformed points x~_i = (arccos gamma(r_i), theta_i, phi_i)
 * (eq. x_tilde) with rho of eq. nfsglft_rho, bins them into grid tiles,
 * builds the conversion tables (in long double on the host) and the
 * deconvolution factors, and allocates the workspace.
 *   out        : receives the plan handle (host pointer)
 *   p          : parameters (host pointer)
 *   M          : number of points, 1 <= M < 2^31
 *   points_dev : device pointer, M x 3 (double or float by p->precision);
 *                may be freed once sgl_plan returns
 *   hip_stream : hipStream_t used by every later call; NULL = null stream
 * Synchronous.  Errors: SGL_E_INVAL (null pointers, bad parameters, NaN/Inf
 * points), SGL_E_RANGE (p->rho > 0 but below max |x_i|), SGL_E_UNSUPPORTED,
 * SGL_E_NOMEM, SGL_E_DEVICE.  On error *out is set to NULL. */
sgl_status sgl_plan(sgl_plan_t *out, const sgl_params *p, int64_t M, const void *points_dev,
                    void *hip_stream);

/* f = Lambda fhat, approximately (Thm. 6.2 with the NFFT; exactly up to
 * rounding with SGL_FLAG_EXACT_NDFT).
 *   fhat_dev : Nc complex, coefficient order mu (input, not modified)
 *   f_dev    : M complex, caller's point order (output, overwritten) */
sgl_status sgl_forward(sgl_plan_t plan, const void *fhat_dev, void *f_dev);

/* fhat = Lambda^H f (Cor. 6.3): exact adjoint of the fast forward.
 *   f_dev    : M complex, caller's point order (input, not modified)
 *   fhat_dev : Nc complex, order mu (output, overwritten) */
sgl_status sgl_adjoint(sgl_plan_t plan, const void *f_dev, void *fhat_dev);

/* Stage: the conversion alone (all factors of Thm. 6.2 right of N):
 * fhat (Nc complex) -> eta on the reduced grid (see sgl_eta_dims). */
sgl_status sgl_conv_forward(sgl_plan_t plan, const void *fhat_dev, void *eta_dev);

/* Stage: adjoint of sgl_conv_forward (Cor. 6.3 without N^H). */
sgl_status sgl_conv_adjoint(sgl_plan_t plan, const void *eta_dev, void *fhat_dev);

/* Stage: the 3D NFFT of Section 2 (or the NDFT with SGL_FLAG_EXACT_NDFT)
 * alone, evaluating p(x~_i) = sum_k eta_k e^{i <k, x~_i>} at the plan's
 * transformed points: eta (reduced grid) -> f (M complex, caller's order). */
sgl_status sgl_nfft_forward(sgl_plan_t plan, const void *eta_dev, void *f_dev);

/* Stage: adjoint of sgl_nfft_forward: f (M complex) -> eta (reduced grid). */
sgl_status sgl_nfft_adjoint(sgl_plan_t plan, const void *f_dev, void *eta_dev);

/* Gradient with respect to the point positions (rho held fixed) of a real
 * loss L(f), f = Lambda fhat (Def. 1.3), given g = dL/d conj(f):
 *   grad[3i + c] = Re(conj(g_i) d f_i / d x_ic),
 * the conjugate-Wirtinger convention (the gradient with respect to fhat is
 * sgl_adjoint(g)).  f_i is the NFFT approximation of Section 2, so the window
 * derivative d/du exp(-(u - l)^2 / (2 lambda)) = -((u - l) / lambda) exp(...)
 * replaces the window, chained through x -> (r, theta, phi) -> x~ (eq. x_tilde)
 * -> u = N x~ / (2 pi).  fhat_dev: Nc complex; points_dev: the M x 3 points the
 * plan was made with (caller order, plan precision); g_dev: M complex; grad_dev:
 * M x 3 reals (plan precision), caller order.  At r = rho (x~_0 = 0: the
 * outermost point when the plan's rho is max |x|, eq. nfsglft_rho) the radial
 * factor takes its limit through the second window derivative, since f
 * depends on x~_0 only through cos x~_0 (the radial expansion of Section 6 is
 * a cosine series).  Points on the z axis or at the origin get NaN (the
 * angles of eq. x_tilde are not differentiable there).  SGL_E_UNSUPPORTED with SGL_FLAG_EXACT_NDFT; SGL_E_INVAL for null or
 * overlapping grad_dev.  Enqueued on the plan's stream. */
sgl_status sgl_grad_points(sgl_plan_t plan, const void *fhat_dev, const void *points_dev, const void *g_dev,
                           void *grad_dev);

/* Inverse transform (the iNFSGLFT of Section 8 over the normal equations of
 * the first kind, Section 2): weighted CGNR (Golub & Van Loan, Alg. 10.4.1)
 * for min_fhat sum_i w_i |y_i - (Lambda fhat)_i|^2, i.e.
 * Lambda^H W Lambda fhat = Lambda^H W y.  y_dev: M complex samples (caller
 * order); w_dev: M nonnegative reals (plan precision) or NULL for W = I
 * (density-compensation weights act as a preconditioner); fhat_dev: Nc
 * complex, the initial guess on entry and the solution on return.  Stops after
 * maxiter iterations or once |Lambda^H W r| <= tol |Lambda^H W y|.  Every
 * iteration runs one forward and one adjoint transform; vectors are in the
 * plan's precision, all scalars in FP64.  info (host, 3 doubles, may be
 * NULL): {iterations, |Lambda^H W r| / |Lambda^H W y|, |W^(1/2) r|}.
 * Synchronous (the step lengths are read on the host each iteration).
 * SGL_E_INVAL for null y/fhat, negative maxiter or tol, or fhat overlapping
 * y or w. */
sgl_status sgl_cgnr(sgl_plan_t plan, const void *y_dev, const void *w_dev, void *fhat_dev, int32_t maxiter,
                    double tol, double *info);

/* Inverse transform for fewer samples than coefficients (M < Nc): the
 * normal equations of the second kind of Section 2, Lambda Lambda^H g = y with
 * fhat = Lambda^H g, by CGNE (Golub & Van Loan, Alg. 10.4.2): the
 * minimum-norm fhat with Lambda fhat = y when the rows of Lambda are
 * independent and the iteration starts in the range of Lambda^H (e.g. from
 * zero).  y_dev: M complex samples (caller order); fhat_dev: Nc complex, the
 * initial guess on entry and the solution on return.  Stops after maxiter
 * iterations or once |y - Lambda fhat| <= tol |y|.  One forward and one
 * adjoint transform per iteration; vectors in the plan's precision, scalars in
 * FP64, reductions in a fixed order.  info (host, 3 doubles, may be NULL):
 * {iterations, |y - Lambda fhat| / |y|, |fhat|}.  Synchronous.  SGL_E_INVAL
 * for null y/fhat, negative maxiter or tol, or fhat overlapping y. */
sgl_status sgl_cgne(sgl_plan_t plan, const void *y_dev, void *fhat_dev, int32_t maxiter, double tol, double *info);

/* ---- Batches of transforms -------------------------------------------------
 * A batch records the forward (fhat_dev[j] -> f_dev[j]) and/or the adjoint
 * (y_dev[j] -> ghat_dev[j]) of n plans (any mix of B, M and precision) once,
 * as one HIP graph whose plans run on nstreams (1..16) concurrent branches
 * (plan j on branch j mod nstreams); sgl_batch_run replays the whole graph with
 * one launch on `stream`.  Each result equals that plan's own sgl_forward /
 * sgl_adjoint on the same buffers, so a batch runs many transforms
 * of the same shapes with no host work between them.
 *   - the pointer arrays are read at creation: the graph keeps the device
 *     addresses, so later runs read whatever those buffers then hold;
 *   - pass NULL for both fhat_dev and f_dev (or y_dev and ghat_dev) to leave
 *     that direction out; not both;
 *   - the plans must be distinct, on the current device, with profiling off,
 *     and must outlive the batch; while a batch runs, do not use its plans
 *     (they share workspace with it);
 *   - output buffers of different plans must not overlap.
 * sgl_batch_create returns SGL_E_INVAL for a violated rule before any device
 * work, and SGL_E_DEVICE if the capture fails.  sgl_batch_destroy waits for
 * `stream` first. */
typedef struct sgl_batch_s *sgl_batch_t;
sgl_status sgl_batch_create(sgl_batch_t *out, const sgl_plan_t *plans, int32_t n, const void *const *fhat_dev,
                            void *const *f_dev, const void *const *y_dev, void *const *ghat_dev, int32_t nstreams,
                            void *stream);
sgl_status sgl_batch_run(sgl_batch_t batch);
sgl_status sgl_batch_destroy(sgl_batch_t batch);

/* ---- Learned density-compensation weights for sgl_cgnr -------------------
 * Weights w_i = exp(c_i - d_i - |x_i|^2) / M, with d_i the log point density
 * in Cartesian cells of edge rho / 16 and c = MLP(features): a 4 -> 64 -> 64
 * -> 1 tanh network (float32 parameters, sgl_mlp_num_params() of them:
 * W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3).  With c = 0 (c_dev NULL)
 * the weights are the plain histogram estimate e^{-r^2} / (M density), the
 * quadrature weights of the e^{-r^2}-orthonormal SGL basis; the network is
 * trained to improve on them (the training loop is in the Python binding).
 * All calls enqueue on the plan's stream; SGL_E_INVAL for null pointers. */
int32_t sgl_mlp_num_params(void);
/* feat_dev: M x 4 floats {log density at cell edges rho/32, rho/16, rho/8; |x|^2 / rho^2};
 * points_dev: the plan's M x 3 points (plan precision).  Synchronous. */
sgl_status sgl_point_features(sgl_plan_t plan, const void *points_dev, float *feat_dev);
/* c_dev[i] = MLP(feat_i) (M floats). */
sgl_status sgl_mlp_forward(sgl_plan_t plan, const float *params_dev, const float *feat_dev, float *c_dev);
/* grad_dev = d/dparams sum_i dc_i MLP(feat_i) (sgl_mlp_num_params floats);
 * deterministic (fixed-order reduction).  Synchronous. */
sgl_status sgl_mlp_backward(sgl_plan_t plan, const float *params_dev, const float *feat_dev, const float *dc_dev,
                            float *grad_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * sgl_mlp_backward with its per-block partial gradients (128 points a block)
 * kept in a fixed device array of the library instead of a per-call
 * allocation.  The array holds SGL_MLP_NOALLOC_MAX_POINTS / 128 blocks of
 * sgl_mlp_num_params floats (46.5 MB on every device the call runs on, held
 * until the process ends).  Same result as sgl_mlp_backward, bit for bit.
 * Allocates nothing, does not synchronise: enqueued on the plan's stream.
 * The first call on a device looks up the array's address on that device.
 * SGL_E_UNSUPPORTED for plans with more than SGL_MLP_NOALLOC_MAX_POINTS
 * points; SGL_E_INVAL for null arguments.  Every call on one device shares
 * the array: calls that overlap in time on one device (two streams, two host
 * threads) race and return wrong gradients. */
#define SGL_MLP_NOALLOC_MAX_POINTS 327680
sgl_status sgl_mlp_backward_noalloc(sgl_plan_t plan, const float *params_dev, const float *feat_dev,
                                    const float *dc_dev, float *grad_dev);
/* One Adam step (Kingma & Ba) on the parameters; m_dev, v_dev: moment buffers
 * (start at zero), step >= 1. */
sgl_status sgl_mlp_adam(sgl_plan_t plan, float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                        float lr, float beta1, float beta2, float eps, int32_t step);
/* w_dev: M weights (plan precision) from c (NULL: c = 0) and the features. */
sgl_status sgl_mlp_weights(sgl_plan_t plan, const float *c_dev, const float *feat_dev, void *w_dev);
/* dc_dev[i] = scale * 2 Re(y_i conj(g_i)) w_i: the gradient with respect to c of
 * scale * |Lambda^H (w y) - fhat|^2 when g = Lambda (Lambda^H (w y) - fhat). */
sgl_status sgl_mlp_weight_grad(sgl_plan_t plan, const void *y_dev, const void *g_dev, const void *w_dev,
                               double scale, float *dc_dev);

/* One training step (synchronous) on nbatch coefficient vectors fhat_dev
 * (nbatch x num_coeffs, plan precision, drawn by the caller): with y = Lambda
 * fhat_b and w from the current network, the loss is the mean over b of
 * |Lambda^H (w y) - fhat_b|^2 / |fhat_b|^2, i.e. how far Lambda^H W Lambda is
 * from the identity on those vectors.  Its gradient goes through the network
 * (sgl_mlp_weight_grad, sgl_mlp_backward) into one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8, learning rate lr, step >= 1).  *loss: the loss
 * before the update.  Allocates its workspace; SGL_E_INVAL for null pointers,
 * nbatch < 1 or a zero coefficient vector. */
sgl_status sgl_mlp_train_step(sgl_plan_t plan, float *params_dev, float *m_dev, float *v_dev, const float *feat_dev,
                              const void *fhat_dev, int32_t nbatch, float lr, int32_t step, double *loss);

/* Forward f = Lambda fhat and adjoint ghat = Lambda^H y in one call, the two
 * running concurrently: the forward on the plan's stream, the adjoint on a
 * second stream of the plan with scratch of its own (allocated on the first
 * call, about the size of the plan's FFT buffers; freed by sgl_destroy).  The
 * plan's stream waits for both before later work.  Results equal those of
 * sgl_forward and sgl_adjoint.  With profiling on (sgl_plan_profile) both run
 * on the plan's stream, one after the other.  No buffer may overlap another
 * (SGL_E_INVAL). */
sgl_status sgl_forward_adjoint(sgl_plan_t plan, const void *fhat_dev, void *f_dev, const void *y_dev,
                               void *ghat_dev);

/* The rho the plan uses (host pointer out): the user's rho, or max_i |x_i|
 * (eq. nfsglft_rho, Section 8) when the plan was made with rho <= 0, or 1 when
 * every point is at the origin (then only l = 0 terms are nonzero and any
 * rho > 0 is exact).  SGL_E_INVAL for a null plan or rho. */
sgl_status sgl_plan_rho(sgl_plan_t plan, double *rho);

/* Informational: number of points, FFT grid sigma*n, stored (pruned) grid
 * extents, gather tile edges, and bytes of device workspace.  info must
 * hold 12 int64 values: {M, N0, N1, N2, E0, E1, E2, L0, L1, L2, bytes,
 * gather_mode (0 = LDS tiles, 1 = wide windows: the box streamed through LDS
 * in slabs for the gather, cell-owned blocks for the scatter,
 * 2 = LDS tiles with the FP16 hi/lo matrix-core gather and spread of FP32
 * plans, 3 = LDS tiles with the FP64 matrix-core spread of FP64 plans)}. */
sgl_status sgl_plan_info(sgl_plan_t plan, int64_t info[12]);

/* Stages timed by the optional per-stage profiler (forward: radial and polar
 * conversion, FFT passes A (along m), B (along k1), C (along k0), gather;
 * adjoint: scatter, FFT passes C, B, A, polar and radial adjoint conversion;
 * exact mode: NDFT and its adjoint; fold: summation of the staged window
 * boxes of the tiled scatter into the grid). */
enum {
  SGL_STAGE_CONV_RADIAL = 0,
  SGL_STAGE_CONV_POLAR,
  SGL_STAGE_FFT_A,
  SGL_STAGE_FFT_B,
  SGL_STAGE_FFT_C,
  SGL_STAGE_GATHER,
  SGL_STAGE_SCATTER,
  SGL_STAGE_FFT_CH,
  SGL_STAGE_FFT_BH,
  SGL_STAGE_FFT_AH,
  SGL_STAGE_CONV_POLAR_ADJ,
  SGL_STAGE_CONV_RADIAL_ADJ,
  SGL_STAGE_NDFT,
  SGL_STAGE_NDFT_ADJ,
  SGL_STAGE_FOLD,
  SGL_NUM_STAGES
};

/* Enable (1) or disable (0) per-stage timing: while enabled, every kernel
 * launch of the plan is bracketed by HIP events recorded on the plan's
 * stream.  Enabling allocates the events (SGL_E_NOMEM / SGL_E_DEVICE). */
sgl_status sgl_plan_profile(sgl_plan_t plan, int32_t enable);

/* Wait for the plan's stream and return, per stage, the summed event time in
 * milliseconds and the number of launches since the last reset (host arrays
 * of SGL_NUM_STAGES entries).  reset != 0 zeroes the totals afterwards. */
sgl_status sgl_plan_stage_times(sgl_plan_t plan, double ms[SGL_NUM_STAGES], int64_t counts[SGL_NUM_STAGES],
                                int32_t reset);

/* Release the plan and its device memory (waits for its stream).  Ends the
 * lifetime that sgl_plan began: the point transform, bins, tables and
 * workspace of the precomputation of Section 6 (Thm. 6.2: everything that
 * does not depend on fhat or y).  NULL is SGL_E_INVAL. */
sgl_status sgl_destroy(sgl_plan_t plan);

/* Name and description of the last HIP error this thread's calls turned into
 * SGL_E_DEVICE or SGL_E_NOMEM (empty if none); valid until the next such error. */
const char *sgl_last_error(void);

/* Static description of a status code (not a passage of the paper: the
 * codes are this library's error model; unknown codes give "unknown status"). */
const char *sgl_status_string(sgl_status s);

#ifdef __cplusplus
}
#endif

#endif /* SGL_H */
