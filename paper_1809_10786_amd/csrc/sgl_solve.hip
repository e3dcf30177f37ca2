// Weighted CGNR for the inverse transform (Section 2, normal equations of the
// first kind, and the iNFSGLFT of Section 8): the least-squares solution of
//   min_fhat sum_i w_i |y_i - (Lambda fhat)_i|^2,
// i.e. Lambda^H W Lambda fhat = Lambda^H W y, by the CGLS form of the conjugate
// gradient method (Golub & Van Loan, Alg. 10.4.1).  Every iteration is one
// forward and one adjoint transform of the plan; the vectors live in the
// plan's precision, every scalar (inner products, alpha, beta, residual norms)
// is accumulated and kept in FP64 (the paper computed alpha and beta in
// extended precision).  Inner products are reduced in a fixed order (block
// partials, then one block), so runs are deterministic.  The step lengths
// stay on the device: the host reads the solver state every kCheck
// iterations, and iterations past convergence change nothing, so the count is
// exact.  W = I when no weights
// are given; density-compensation weights make Lambda^H W Lambda closer to the
// identity (the SGL functions are orthonormal for the weight e^{-r^2}), which
// is their role as a preconditioner.
#include <algorithm>
#include <cmath>

#include "sgl_internal.h"

namespace sgl {

namespace {

constexpr int kRedBlocks = 512;

// partial[b] = sum over the block's indices of w_i Re(conj(a_i) b_i)
template <class R>
__global__ __launch_bounds__(256) void k_dot_partial(const cplx<R> *__restrict__ a, const cplx<R> *__restrict__ b,
                                                     const R *__restrict__ w, int64_t n,
                                                     double *__restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double v = (double)a[i].re * (double)b[i].re + (double)a[i].im * (double)b[i].im;
    if (w) v *= (double)w[i];
    s += v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dot_final(const double *__restrict__ partial, int n,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Device-resident scalars of one solve (FP64): the step lengths never leave
// the device; the host reads the state once every kCheck iterations.
enum { kGamma = 0, kGammaRef, kDelta, kAlpha, kBeta, kDone, kIter, kTol2, kNew, kNumScalars };
constexpr int kCheck = 8;

// y += sign * sc[kAlpha] x
template <class R>
__global__ __launch_bounds__(256) void k_axpy(cplx<R> *__restrict__ y, const cplx<R> *__restrict__ x,
                                              const double *__restrict__ sc, double sign, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  const double alpha = sign * sc[kAlpha];
  if (i < n) y[i] = cplx<R>{(R)((double)y[i].re + alpha * x[i].re), (R)((double)y[i].im + alpha * x[i].im)};
}

// p = s + sc[kBeta] p
template <class R>
__global__ __launch_bounds__(256) void k_xpby(cplx<R> *__restrict__ p, const cplx<R> *__restrict__ s,
                                              const double *__restrict__ sc, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  const double beta = sc[kBeta];
  if (i < n) p[i] = cplx<R>{(R)(s[i].re + beta * p[i].re), (R)(s[i].im + beta * p[i].im)};
}

// out = w (a - b)   (w = 1 when absent)
template <class R>
__global__ __launch_bounds__(256) void k_wsub(cplx<R> *__restrict__ out, const cplx<R> *__restrict__ a,
                                              const cplx<R> *__restrict__ b, const R *__restrict__ w, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const R s = w ? w[i] : (R)1;
  out[i] = cplx<R>{s * (a[i].re - b[i].re), s * (a[i].im - b[i].im)};
}

// out = w a
template <class R>
__global__ __launch_bounds__(256) void k_wmul(cplx<R> *__restrict__ out, const cplx<R> *__restrict__ a,
                                              const R *__restrict__ w, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const R s = w ? w[i] : (R)1;
  out[i] = cplx<R>{s * a[i].re, s * a[i].im};
}

// CG step lengths on the device.  An iteration after convergence (or after a
// zero denominator) has alpha = 0 and leaves x and r unchanged, so the host
// may launch several iterations between its checks.
//   alpha = num / den (num = sc[num_idx], den = sc[kDelta])
__global__ void k_cg_alpha(double *sc, int num_idx) {
  const double den = sc[kDelta];
  if (sc[kDone] == 0.0 && !(den > 0.0)) sc[kDone] = 1.0;
  sc[kAlpha] = sc[kDone] == 0.0 ? sc[num_idx] / den : 0.0;
}
//   beta = new / old (new = sc[kNew], old = sc[num_idx]), then the stopping
//   test sc[num_idx] <= tol^2 sc[kGammaRef] on the new value
__global__ void k_cg_beta(double *sc, int num_idx) {
  if (sc[kDone] != 0.0) {
    sc[kBeta] = 0.0;
    return;
  }
  const double nw = sc[kNew];
  sc[kBeta] = sc[num_idx] > 0.0 ? nw / sc[num_idx] : 0.0;
  sc[num_idx] = nw;
  sc[kIter] += 1.0;
  if (nw <= sc[kTol2] * sc[kGammaRef]) sc[kDone] = 1.0;
}
__global__ void k_set_scalar(double *sc, int idx, double v) { sc[idx] = v; }

//   before the first iteration: done if the reference is zero or the start
//   already meets the tolerance
__global__ void k_cg_start(double *sc, int num_idx) {
  sc[kIter] = 0.0;
  sc[kDone] = (sc[kGammaRef] > 0.0 && sc[num_idx] > sc[kTol2] * sc[kGammaRef]) ? 0.0 : 1.0;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class R>
struct Solver {
  Plan &p;
  const cplx<R> *y;
  const R *w;
  cplx<R> *x;
  cplx<R> *r, *q, *t;  // M: residual, Lambda p, weighted vectors
  cplx<R> *s, *pv;     // Nc: normal residual, search direction
  double *partial, *sc;
  int64_t M, nc;

  // sc[idx] = sum_i w_i Re(conj(a_i) b_i), fixed-order reduction on the device
  void dot(const cplx<R> *a, const cplx<R> *b, const R *ww, int64_t n, int idx) {
    const int nb = (int)std::min<int64_t>(kRedBlocks, (n + 255) / 256);
    k_dot_partial<R><<<nb, 256, 0, p.stream>>>(a, b, ww, n, partial);
    k_dot_final<<<1, 256, 0, p.stream>>>(partial, nb, sc + idx);
  }
  // host copy of the scalars (waits for the stream)
  hipError_t read(double *h) {
    hipError_t e = hipMemcpyAsync(h, sc, kNumScalars * sizeof(double), hipMemcpyDeviceToHost, p.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
    return e == hipSuccess ? hipGetLastError() : e;
  }
  hipError_t set(int idx, double v) {
    k_set_scalar<<<1, 1, 0, p.stream>>>(sc, idx, v);
    return hipGetLastError();
  }
};

}  // namespace

#define CG_TRY_ST(x)             \
  do {                           \
    st = (x);                    \
    if (st != SGL_OK) goto done; \
  } while (0)
#define CG_TRY_HIP(x)               \
  do {                              \
    e = (x);                        \
    if (e != hipSuccess) goto done; \
  } while (0)

template <class R>
static sgl_status cgnr_typed(Plan &p, const void *y_dev, const void *w_dev, void *fhat_dev, int maxiter, double tol,
                             double *info, sgl_status (*fwd)(Plan &, const void *, void *),
                             sgl_status (*adj)(Plan &, const void *, void *)) {
  Solver<R> S{p};
  S.y = (const cplx<R> *)y_dev;
  S.w = (const R *)w_dev;
  S.x = (cplx<R> *)fhat_dev;
  S.M = p.M;
  S.nc = (int64_t)p.B * (p.B + 1) * (2 * p.B + 1) / 6;
  void *ws = nullptr;
  const size_t cb = sizeof(cplx<R>);
  const size_t bytes = 3 * (size_t)S.M * cb + 2 * (size_t)S.nc * cb + (kRedBlocks + kNumScalars) * sizeof(double);
  if (hipMalloc(&ws, bytes) != hipSuccess) return SGL_E_NOMEM;
  char *b = (char *)ws;
  S.r = (cplx<R> *)b;
  S.q = S.r + S.M;
  S.t = S.q + S.M;
  S.s = S.t + S.M;
  S.pv = S.s + S.nc;
  S.partial = (double *)(S.pv + S.nc);
  S.sc = S.partial + kRedBlocks;
  sgl_status st = SGL_OK;
  hipError_t e = hipSuccess;
  double h[kNumScalars] = {0};
  int launched = 0;
  // stopping test on the squared norms: |Lambda^H W r|^2 <= tol^2 |Lambda^H W y|^2
  CG_TRY_HIP(S.set(kTol2, tol * tol));
  // reference: |Lambda^H W y|^2 for the relative normal-equation residual
  k_wmul<R><<<blocks(S.M), 256, 0, p.stream>>>(S.t, S.y, S.w, S.M);
  CG_TRY_ST(adj(p, S.t, S.s));
  S.dot(S.s, S.s, nullptr, S.nc, kGammaRef);
  // r = y - Lambda x, s = Lambda^H W r, p = s
  CG_TRY_ST(fwd(p, S.x, S.q));
  k_wsub<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.y, S.q, nullptr, S.M);
  k_wmul<R><<<blocks(S.M), 256, 0, p.stream>>>(S.t, S.r, S.w, S.M);
  CG_TRY_ST(adj(p, S.t, S.s));
  CG_TRY_HIP(hipMemcpyAsync(S.pv, S.s, S.nc * cb, hipMemcpyDeviceToDevice, p.stream));
  S.dot(S.s, S.s, nullptr, S.nc, kGamma);
  k_cg_start<<<1, 1, 0, p.stream>>>(S.sc, kGamma);
  CG_TRY_HIP(S.read(h));
  while (launched < maxiter && h[kDone] == 0.0) {
    const int n = std::min(kCheck, maxiter - launched);
    for (int k = 0; k < n; ++k) {
      CG_TRY_ST(fwd(p, S.pv, S.q));                                   // q = Lambda p
      S.dot(S.q, S.q, S.w, S.M, kDelta);                              // delta = q^H W q
      k_cg_alpha<<<1, 1, 0, p.stream>>>(S.sc, kGamma);                // alpha = gamma / delta
      k_axpy<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.x, S.pv, S.sc, 1.0, S.nc);   // x += alpha p
      k_axpy<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.q, S.sc, -1.0, S.M);     // r -= alpha q
      k_wmul<R><<<blocks(S.M), 256, 0, p.stream>>>(S.t, S.r, S.w, S.M);
      CG_TRY_ST(adj(p, S.t, S.s));                                    // s = Lambda^H W r
      S.dot(S.s, S.s, nullptr, S.nc, kNew);
      k_cg_beta<<<1, 1, 0, p.stream>>>(S.sc, kGamma);                 // beta = gnew / gamma
      k_xpby<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.pv, S.s, S.sc, S.nc);        // p = s + beta p
    }
    launched += n;
    CG_TRY_HIP(S.read(h));
  }
  S.dot(S.r, S.r, S.w, S.M, kNew);  // |W^(1/2) r|^2
  CG_TRY_HIP(S.read(h));
done:
  (void)hipStreamSynchronize(p.stream);
  (void)hipFree(ws);
  if (st != SGL_OK) return st;
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SGL_E_NOMEM : SGL_E_DEVICE;
  if (info) {
    info[0] = h[kIter];
    info[1] = h[kGammaRef] > 0.0 ? std::sqrt(h[kGamma] / h[kGammaRef]) : 0.0;  // |Lambda^H W r| / |Lambda^H W y|
    info[2] = std::sqrt(h[kNew]);                                             // |W^(1/2) r|
  }
  return SGL_OK;
}

sgl_status cgnr_run(Plan &p, const void *y_dev, const void *w_dev, void *fhat_dev, int maxiter, double tol,
                    double *info, sgl_status (*fwd)(Plan &, const void *, void *),
                    sgl_status (*adj)(Plan &, const void *, void *)) {
  return p.prec == SGL_F64 ? cgnr_typed<double>(p, y_dev, w_dev, fhat_dev, maxiter, tol, info, fwd, adj)
                           : cgnr_typed<float>(p, y_dev, w_dev, fhat_dev, maxiter, tol, info, fwd, adj);
}

// CGNE (Golub & Van Loan, Alg. 10.4.2; Craig's method) for the normal
// equations of the second kind of an under-determined system (Section 2):
// Lambda Lambda^H g = y, fhat = Lambda^H g, the minimum-norm solution when
// the iteration starts from fhat in the range of Lambda^H (e.g. zero).  In
// terms of fhat: r = y - Lambda fhat, p = Lambda^H r, then per iteration
//   alpha = |r|^2 / |p|^2,  fhat += alpha p,  r -= alpha Lambda p,
//   beta = |r_new|^2 / |r|^2,  p = Lambda^H r + beta p.
template <class R>
static sgl_status cgne_typed(Plan &p, const void *y_dev, void *fhat_dev, int maxiter, double tol, double *info,
                             sgl_status (*fwd)(Plan &, const void *, void *),
                             sgl_status (*adj)(Plan &, const void *, void *)) {
  Solver<R> S{p};
  S.y = (const cplx<R> *)y_dev;
  S.w = nullptr;
  S.x = (cplx<R> *)fhat_dev;
  S.M = p.M;
  S.nc = (int64_t)p.B * (p.B + 1) * (2 * p.B + 1) / 6;
  void *ws = nullptr;
  const size_t cb = sizeof(cplx<R>);
  const size_t bytes = 2 * (size_t)S.M * cb + 2 * (size_t)S.nc * cb + (kRedBlocks + kNumScalars) * sizeof(double);
  if (hipMalloc(&ws, bytes) != hipSuccess) return SGL_E_NOMEM;
  char *b = (char *)ws;
  S.r = (cplx<R> *)b;
  S.q = S.r + S.M;
  S.s = S.q + S.M;
  S.pv = S.s + S.nc;
  S.t = nullptr;
  S.partial = (double *)(S.pv + S.nc);
  S.sc = S.partial + kRedBlocks;
  sgl_status st = SGL_OK;
  hipError_t e = hipSuccess;
  double h[kNumScalars] = {0};
  int launched = 0;
  CG_TRY_HIP(S.set(kTol2, tol * tol));
  S.dot(S.y, S.y, nullptr, S.M, kGammaRef);  // |y|^2
  // r = y - Lambda x, p = Lambda^H r
  CG_TRY_ST(fwd(p, S.x, S.q));
  k_wsub<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.y, S.q, nullptr, S.M);
  CG_TRY_ST(adj(p, S.r, S.pv));
  S.dot(S.r, S.r, nullptr, S.M, kGamma);  // |r|^2
  k_cg_start<<<1, 1, 0, p.stream>>>(S.sc, kGamma);
  CG_TRY_HIP(S.read(h));
  while (launched < maxiter && h[kDone] == 0.0) {
    const int n = std::min(kCheck, maxiter - launched);
    for (int k = 0; k < n; ++k) {
      S.dot(S.pv, S.pv, nullptr, S.nc, kDelta);                     // |p|^2
      k_cg_alpha<<<1, 1, 0, p.stream>>>(S.sc, kGamma);              // alpha = |r|^2 / |p|^2
      k_axpy<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.x, S.pv, S.sc, 1.0, S.nc);   // x += alpha p
      CG_TRY_ST(fwd(p, S.pv, S.q));                                 // q = Lambda p
      k_axpy<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.q, S.sc, -1.0, S.M);     // r -= alpha q
      S.dot(S.r, S.r, nullptr, S.M, kNew);
      k_cg_beta<<<1, 1, 0, p.stream>>>(S.sc, kGamma);               // beta = |r_new|^2 / |r|^2
      CG_TRY_ST(adj(p, S.r, S.s));                                  // s = Lambda^H r
      k_xpby<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.pv, S.s, S.sc, S.nc);        // p = s + beta p
    }
    launched += n;
    CG_TRY_HIP(S.read(h));
  }
  S.dot(S.x, S.x, nullptr, S.nc, kNew);  // |fhat|^2
  CG_TRY_HIP(S.read(h));
done:
  (void)hipStreamSynchronize(p.stream);
  (void)hipFree(ws);
  if (st != SGL_OK) return st;
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SGL_E_NOMEM : SGL_E_DEVICE;
  if (info) {
    info[0] = h[kIter];
    info[1] = h[kGammaRef] > 0.0 ? std::sqrt(h[kGamma] / h[kGammaRef]) : 0.0;  // |y - Lambda fhat| / |y|
    info[2] = std::sqrt(h[kNew]);                                             // |fhat|
  }
  return SGL_OK;
}

#undef CG_TRY_ST
#undef CG_TRY_HIP

sgl_status cgne_run(Plan &p, const void *y_dev, void *fhat_dev, int maxiter, double tol, double *info,
                    sgl_status (*fwd)(Plan &, const void *, void *),
                    sgl_status (*adj)(Plan &, const void *, void *)) {
  return p.prec == SGL_F64 ? cgne_typed<double>(p, y_dev, fhat_dev, maxiter, tol, info, fwd, adj)
                           : cgne_typed<float>(p, y_dev, fhat_dev, maxiter, tol, info, fwd, adj);
}

}  // namespace sgl
