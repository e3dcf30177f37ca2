// Weighted CGNR for the inverse transform (Section 2, normal equations of the
// first kind, and the iNFSGLFT of Section 8): the least-squares solution of
//   min_fhat sum_i w_i |y_i - (Lambda fhat)_i|^2,
// i.e. Lambda^H W Lambda fhat = Lambda^H W y, by the CGLS form of the conjugate
// gradient method (Golub & Van Loan, Alg. 10.4.1).  Every iteration is one
// forward and one adjoint transform of the plan; the vectors live in the
// plan's precision, every scalar (inner products, alpha, beta, residual norms)
// is accumulated and kept in FP64 (the paper computed alpha and beta in
// extended precision).  Inner products are reduced in a fixed order (block
// partials, then one block), so runs are deterministic.  W = I when no weights
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

// y += alpha x
template <class R>
__global__ __launch_bounds__(256) void k_axpy(cplx<R> *__restrict__ y, const cplx<R> *__restrict__ x, double alpha,
                                              int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n) y[i] = cplx<R>{(R)((double)y[i].re + alpha * x[i].re), (R)((double)y[i].im + alpha * x[i].im)};
}

// p = s + beta p
template <class R>
__global__ __launch_bounds__(256) void k_xpby(cplx<R> *__restrict__ p, const cplx<R> *__restrict__ s, double beta,
                                              int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
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

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class R>
struct Solver {
  Plan &p;
  const cplx<R> *y;
  const R *w;
  cplx<R> *x;
  cplx<R> *r, *q, *t;  // M: residual, Lambda p, weighted vectors
  cplx<R> *s, *pv;     // Nc: normal residual, search direction
  double *partial, *scalar;
  int64_t M, nc;

  hipError_t dot(const cplx<R> *a, const cplx<R> *b, const R *ww, int64_t n, double *out) {
    const int nb = (int)std::min<int64_t>(kRedBlocks, (n + 255) / 256);
    k_dot_partial<R><<<nb, 256, 0, p.stream>>>(a, b, ww, n, partial);
    k_dot_final<<<1, 256, 0, p.stream>>>(partial, nb, scalar);
    hipError_t e = hipMemcpyAsync(out, scalar, sizeof(double), hipMemcpyDeviceToHost, p.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
    return e == hipSuccess ? hipGetLastError() : e;
  }
};

}  // namespace

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
  const size_t bytes = 3 * (size_t)S.M * cb + 2 * (size_t)S.nc * cb + (kRedBlocks + 1) * sizeof(double);
  if (hipMalloc(&ws, bytes) != hipSuccess) return SGL_E_NOMEM;
  char *b = (char *)ws;
  S.r = (cplx<R> *)b;
  S.q = S.r + S.M;
  S.t = S.q + S.M;
  S.s = S.t + S.M;
  S.pv = S.s + S.nc;
  S.partial = (double *)(S.pv + S.nc);
  S.scalar = S.partial + kRedBlocks;
  sgl_status st = SGL_OK;
  hipError_t e = hipSuccess;
  double gamma = 0.0, gamma_ref = 0.0, delta = 0.0, rr = 0.0;
  int it = 0;
#define CG_TRY_ST(x)          \
  do {                        \
    st = (x);                 \
    if (st != SGL_OK) goto done; \
  } while (0)
#define CG_TRY_HIP(x)                 \
  do {                                \
    e = (x);                          \
    if (e != hipSuccess) goto done;   \
  } while (0)
  // reference: |Lambda^H W y|^2 for the relative normal-equation residual
  k_wmul<R><<<blocks(S.M), 256, 0, p.stream>>>(S.t, S.y, S.w, S.M);
  CG_TRY_ST(adj(p, S.t, S.s));
  CG_TRY_HIP(S.dot(S.s, S.s, nullptr, S.nc, &gamma_ref));
  // r = y - Lambda x, s = Lambda^H W r, p = s
  CG_TRY_ST(fwd(p, S.x, S.q));
  k_wsub<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.y, S.q, nullptr, S.M);
  k_wmul<R><<<blocks(S.M), 256, 0, p.stream>>>(S.t, S.r, S.w, S.M);
  CG_TRY_ST(adj(p, S.t, S.s));
  CG_TRY_HIP(hipMemcpyAsync(S.pv, S.s, S.nc * cb, hipMemcpyDeviceToDevice, p.stream));
  CG_TRY_HIP(S.dot(S.s, S.s, nullptr, S.nc, &gamma));
  while (it < maxiter && gamma_ref > 0.0 && std::sqrt(gamma / gamma_ref) > tol) {
    CG_TRY_ST(fwd(p, S.pv, S.q));                                   // q = Lambda p
    CG_TRY_HIP(S.dot(S.q, S.q, S.w, S.M, &delta));                  // delta = q^H W q
    if (!(delta > 0.0)) break;
    const double alpha = gamma / delta;
    k_axpy<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.x, S.pv, alpha, S.nc);   // x += alpha p
    k_axpy<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.q, -alpha, S.M);     // r -= alpha q
    k_wmul<R><<<blocks(S.M), 256, 0, p.stream>>>(S.t, S.r, S.w, S.M);
    CG_TRY_ST(adj(p, S.t, S.s));                                    // s = Lambda^H W r
    double gnew = 0.0;
    CG_TRY_HIP(S.dot(S.s, S.s, nullptr, S.nc, &gnew));
    const double beta = gnew / gamma;
    gamma = gnew;
    k_xpby<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.pv, S.s, beta, S.nc);    // p = s + beta p
    ++it;
  }
  CG_TRY_HIP(S.dot(S.r, S.r, S.w, S.M, &rr));
done:
#undef CG_TRY_ST
#undef CG_TRY_HIP
  hipStreamSynchronize(p.stream);
  hipFree(ws);
  if (st != SGL_OK) return st;
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SGL_E_NOMEM : SGL_E_DEVICE;
  if (info) {
    info[0] = it;
    info[1] = gamma_ref > 0.0 ? std::sqrt(gamma / gamma_ref) : 0.0;  // |Lambda^H W r| / |Lambda^H W y|
    info[2] = std::sqrt(rr);                                          // |W^(1/2) r|
  }
  return SGL_OK;
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
  const size_t bytes = 2 * (size_t)S.M * cb + 2 * (size_t)S.nc * cb + (kRedBlocks + 1) * sizeof(double);
  if (hipMalloc(&ws, bytes) != hipSuccess) return SGL_E_NOMEM;
  char *b = (char *)ws;
  S.r = (cplx<R> *)b;
  S.q = S.r + S.M;
  S.s = S.q + S.M;
  S.pv = S.s + S.nc;
  S.t = nullptr;
  S.partial = (double *)(S.pv + S.nc);
  S.scalar = S.partial + kRedBlocks;
  sgl_status st = SGL_OK;
  hipError_t e = hipSuccess;
  double yy = 0.0, rr = 0.0, pp = 0.0, xx = 0.0;
  int it = 0;
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
  CG_TRY_HIP(S.dot(S.y, S.y, nullptr, S.M, &yy));
  // r = y - Lambda x, p = Lambda^H r
  CG_TRY_ST(fwd(p, S.x, S.q));
  k_wsub<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.y, S.q, nullptr, S.M);
  CG_TRY_ST(adj(p, S.r, S.pv));
  CG_TRY_HIP(S.dot(S.r, S.r, nullptr, S.M, &rr));
  while (it < maxiter && yy > 0.0 && std::sqrt(rr / yy) > tol) {
    CG_TRY_HIP(S.dot(S.pv, S.pv, nullptr, S.nc, &pp));            // |p|^2
    if (!(pp > 0.0)) break;
    const double alpha = rr / pp;
    k_axpy<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.x, S.pv, alpha, S.nc);   // x += alpha p
    CG_TRY_ST(fwd(p, S.pv, S.q));                                   // q = Lambda p
    k_axpy<R><<<blocks(S.M), 256, 0, p.stream>>>(S.r, S.q, -alpha, S.M);     // r -= alpha q
    double rnew = 0.0;
    CG_TRY_HIP(S.dot(S.r, S.r, nullptr, S.M, &rnew));
    const double beta = rnew / rr;
    rr = rnew;
    CG_TRY_ST(adj(p, S.r, S.s));                                    // s = Lambda^H r
    k_xpby<R><<<blocks(S.nc), 256, 0, p.stream>>>(S.pv, S.s, beta, S.nc);    // p = s + beta p
    ++it;
  }
  CG_TRY_HIP(S.dot(S.x, S.x, nullptr, S.nc, &xx));
done:
#undef CG_TRY_ST
#undef CG_TRY_HIP
  hipStreamSynchronize(p.stream);
  hipFree(ws);
  if (st != SGL_OK) return st;
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SGL_E_NOMEM : SGL_E_DEVICE;
  if (info) {
    info[0] = it;
    info[1] = yy > 0.0 ? std::sqrt(rr / yy) : 0.0;  // |r| / |y|
    info[2] = std::sqrt(xx);                        // |fhat|
  }
  return SGL_OK;
}

sgl_status cgne_run(Plan &p, const void *y_dev, void *fhat_dev, int maxiter, double tol, double *info,
                    sgl_status (*fwd)(Plan &, const void *, void *),
                    sgl_status (*adj)(Plan &, const void *, void *)) {
  return p.prec == SGL_F64 ? cgne_typed<double>(p, y_dev, fhat_dev, maxiter, tol, info, fwd, adj)
                           : cgne_typed<float>(p, y_dev, fhat_dev, maxiter, tol, info, fwd, adj);
}

sgl_status cgnr_run(Plan &p, const void *y_dev, const void *w_dev, void *fhat_dev, int maxiter, double tol,
                    double *info, sgl_status (*fwd)(Plan &, const void *, void *),
                    sgl_status (*adj)(Plan &, const void *, void *)) {
  return p.prec == SGL_F64 ? cgnr_typed<double>(p, y_dev, w_dev, fhat_dev, maxiter, tol, info, fwd, adj)
                           : cgnr_typed<float>(p, y_dev, w_dev, fhat_dev, maxiter, tol, info, fwd, adj);
}

}  // namespace sgl
