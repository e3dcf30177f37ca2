// Learned density-compensation weights for the weighted CGNR (the inverse
// transform): a small MLP predicts, from local point-density features, the
// weight of every sample,
//   w_i = exp(c_i - d_i - |x_i|^2) / M,   c = MLP(features),
// with d_i the log point density at the middle histogram scale.  The SGL
// functions are orthonormal for the weight e^{-r^2}, so ideal weights are
// e^{-r_i^2} times the volume each point represents, about 1 / (M density);
// with c = 0 the weights are that histogram estimate, and the network learns
// the corrections.  Kernels:
//  - features: counts of points in Cartesian cells of three sizes (integer
//    histograms, so the counts do not depend on the order of the atomic adds),
//    giving log(count / (M h^3)) per scale, and r^2 / rho^2;
//  - MLP 4 -> 64 -> 64 -> 1 with tanh, inference one thread per point;
//  - backward: per-point backpropagation, per-block parameter gradients
//    reduced in a fixed order (deterministic);
//  - Adam update; weights from c; dL/dc from dL/dw.
// Parameters (float32): W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3.
#include <cmath>
#include <mutex>

#include "sgl_internal.h"

namespace sgl {

namespace {

constexpr int kH = 64;                 // hidden width
constexpr int kF = 4;                  // features
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kF, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kNParams = kOffB3 + 1;
constexpr int kGrid[3] = {64, 32, 16};  // cells per axis over [-rho, rho]^3
constexpr int kBP = 128;               // points per backward block

__device__ inline int cell_of(double v, double rho, int n) {
  int c = (int)floor((v + rho) / (2.0 * rho) * n);
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

template <class T>
__global__ __launch_bounds__(256) void k_hist(const T *__restrict__ xyz, int64_t M, double rho,
                                              int32_t *__restrict__ h0, int32_t *__restrict__ h1,
                                              int32_t *__restrict__ h2) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= M) return;
  const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
  int32_t *h[3] = {h0, h1, h2};
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int n = kGrid[s];
    const int c = (cell_of(x, rho, n) * n + cell_of(y, rho, n)) * n + cell_of(z, rho, n);
    atomicAdd(&h[s][c], 1);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_features(const T *__restrict__ xyz, int64_t M, double rho,
                                                  const int32_t *__restrict__ h0, const int32_t *__restrict__ h1,
                                                  const int32_t *__restrict__ h2, float *__restrict__ feat) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= M) return;
  const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
  const int32_t *h[3] = {h0, h1, h2};
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int n = kGrid[s];
    const int c = (cell_of(x, rho, n) * n + cell_of(y, rho, n)) * n + cell_of(z, rho, n);
    const double hs = 2.0 * rho / n;
    feat[4 * i + s] = (float)log((double)h[s][c] / ((double)M * hs * hs * hs));
  }
  feat[4 * i + 3] = (float)((x * x + y * y + z * z) / (rho * rho));
}

__device__ inline void mlp_forward(const float *P, const float *x, float *h1, float *h2, float &c) {
  for (int j = 0; j < kH; ++j) {
    float s = P[kOffB1 + j];
#pragma unroll
    for (int f = 0; f < kF; ++f) s += P[kOffW1 + j * kF + f] * x[f];
    h1[j] = tanhf(s);
  }
  for (int j = 0; j < kH; ++j) {
    float s = P[kOffB2 + j];
    for (int k = 0; k < kH; ++k) s += P[kOffW2 + j * kH + k] * h1[k];
    h2[j] = tanhf(s);
  }
  float s = P[kOffB3];
  for (int j = 0; j < kH; ++j) s += P[kOffW3 + j] * h2[j];
  c = s;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ params, const float *__restrict__ feat,
                                                     int64_t M, float *__restrict__ c) {
  __shared__ float P[kNParams];
  for (int t = threadIdx.x; t < kNParams; t += 256) P[t] = params[t];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= M) return;
  float x[kF], h1[kH], h2[kH], out;
#pragma unroll
  for (int f = 0; f < kF; ++f) x[f] = feat[kF * i + f];
  mlp_forward(P, x, h1, h2, out);
  c[i] = out;
}

// Per block of kBP points: the parameter gradients of sum_i dc_i c_i,
// written to partial[block][kNParams].
__global__ __launch_bounds__(kBP) void k_mlp_backward(const float *__restrict__ params,
                                                      const float *__restrict__ feat,
                                                      const float *__restrict__ dc, int64_t M,
                                                      float *__restrict__ partial) {
  __shared__ float P[kNParams];
  __shared__ float sx[kBP][kF], sd1[kBP][kH + 1], sh1[kBP][kH + 1], sd2[kBP][kH + 1], sh2[kBP][kH + 1];
  __shared__ float sdc[kBP];
  for (int t = threadIdx.x; t < kNParams; t += kBP) P[t] = params[t];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)kBP + threadIdx.x;
  const int p = threadIdx.x;
  float x[kF], h1[kH], h2[kH], out;
  const bool valid = i < M;
#pragma unroll
  for (int f = 0; f < kF; ++f) x[f] = valid ? feat[kF * i + f] : 0.0f;
  mlp_forward(P, x, h1, h2, out);
  const float g = valid ? dc[i] : 0.0f;
  // delta2 = g W3 (1 - h2^2);  delta1 = (W2^T delta2) (1 - h1^2)
  float d2[kH];
  for (int j = 0; j < kH; ++j) d2[j] = g * P[kOffW3 + j] * (1.0f - h2[j] * h2[j]);
  for (int k = 0; k < kH; ++k) {
    float s = 0.0f;
    for (int j = 0; j < kH; ++j) s += P[kOffW2 + j * kH + k] * d2[j];
    sd1[p][k] = s * (1.0f - h1[k] * h1[k]);
    sh1[p][k] = h1[k];
    sd2[p][k] = d2[k];
    sh2[p][k] = h2[k];
  }
#pragma unroll
  for (int f = 0; f < kF; ++f) sx[p][f] = x[f];
  sdc[p] = g;
  __syncthreads();
  // parameter gradients: sums over the block's points in point order
  float *out_p = partial + (size_t)blockIdx.x * kNParams;
  for (int t = threadIdx.x; t < kNParams; t += kBP) {
    float s = 0.0f;
    if (t < kOffB1) {
      const int j = t / kF, f = t % kF;
      for (int q = 0; q < kBP; ++q) s += sd1[q][j] * sx[q][f];
    } else if (t < kOffW2) {
      const int j = t - kOffB1;
      for (int q = 0; q < kBP; ++q) s += sd1[q][j];
    } else if (t < kOffB2) {
      const int j = (t - kOffW2) / kH, k = (t - kOffW2) % kH;
      for (int q = 0; q < kBP; ++q) s += sd2[q][j] * sh1[q][k];
    } else if (t < kOffW3) {
      const int j = t - kOffB2;
      for (int q = 0; q < kBP; ++q) s += sd2[q][j];
    } else if (t < kOffB3) {
      const int j = t - kOffW3;
      for (int q = 0; q < kBP; ++q) s += sdc[q] * sh2[q][j];
    } else {
      for (int q = 0; q < kBP; ++q) s += sdc[q];
    }
    out_p[t] = s;
  }
}

__global__ __launch_bounds__(256) void k_reduce_partials(const float *__restrict__ partial, int nblocks,
                                                         float *__restrict__ grad) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= kNParams) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * kNParams + t];
  grad[t] = (float)s;
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  m[t] = b1 * m[t] + (1.0f - b1) * gt;
  v[t] = b2 * v[t] + (1.0f - b2) * gt * gt;
  p[t] -= lr * (m[t] / c1) / (sqrtf(v[t] / c2) + eps);
}

// w_i = exp(c_i - d_i - r_i^2) / M  (d: feature 1; r^2 = rho^2 feature 3); c may be null (c = 0)
template <class R>
__global__ __launch_bounds__(256) void k_weights(const float *__restrict__ c, const float *__restrict__ feat,
                                                 int64_t M, double rho2, R *__restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= M) return;
  const double ci = c ? (double)c[i] : 0.0;
  w[i] = (R)(exp(ci - (double)feat[kF * i + 1] - rho2 * (double)feat[kF * i + 3]) / (double)M);
}

// dL/dc_i = scale * 2 Re(y_i conj(g_i)) * w_i   (dL/dw_i times dw_i/dc_i = w_i),
// added to dc when accumulate is set
template <class R>
__global__ __launch_bounds__(256) void k_weight_grad(const cplx<R> *__restrict__ y, const cplx<R> *__restrict__ g,
                                                     const R *__restrict__ w, int64_t M, double scale,
                                                     int accumulate, float *__restrict__ dc) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= M) return;
  const float v = (float)(scale * 2.0 * ((double)y[i].re * g[i].re + (double)y[i].im * g[i].im) * (double)w[i]);
  dc[i] = accumulate ? dc[i] + v : v;
}

// out = w a  (real w, complex a)
template <class R>
__global__ __launch_bounds__(256) void k_scale_by(cplx<R> *__restrict__ out, const cplx<R> *__restrict__ a,
                                                  const R *__restrict__ w, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n) out[i] = cplx<R>{w[i] * a[i].re, w[i] * a[i].im};
}

// a -= b
template <class R>
__global__ __launch_bounds__(256) void k_sub_from(cplx<R> *__restrict__ a, const cplx<R> *__restrict__ b,
                                                  int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n) a[i] = cplx<R>{a[i].re - b[i].re, a[i].im - b[i].im};
}

// out[0] = sum |a_i|^2 in FP64, one block, fixed order
template <class R>
__global__ __launch_bounds__(256) void k_norm2(const cplx<R> *__restrict__ a, int64_t n, double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)a[i].re * a[i].re + (double)a[i].im * a[i].im;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int mlp_num_params() { return kNParams; }

hipError_t launch_point_features(const Plan &p, const void *xyz, float *feat) {
  int32_t *h = nullptr;
  const size_t n0 = 64 * 64 * 64, n1 = 32 * 32 * 32, n2 = 16 * 16 * 16;
  hipError_t e = hipMalloc(&h, (n0 + n1 + n2) * sizeof(int32_t));
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(h, 0, (n0 + n1 + n2) * sizeof(int32_t), p.stream);
  if (e == hipSuccess) {
    if (p.prec == SGL_F64) {
      k_hist<double><<<nb(p.M), 256, 0, p.stream>>>((const double *)xyz, p.M, p.rho, h, h + n0, h + n0 + n1);
      k_features<double><<<nb(p.M), 256, 0, p.stream>>>((const double *)xyz, p.M, p.rho, h, h + n0, h + n0 + n1,
                                                        feat);
    } else {
      k_hist<float><<<nb(p.M), 256, 0, p.stream>>>((const float *)xyz, p.M, p.rho, h, h + n0, h + n0 + n1);
      k_features<float><<<nb(p.M), 256, 0, p.stream>>>((const float *)xyz, p.M, p.rho, h, h + n0, h + n0 + n1,
                                                       feat);
    }
    e = hipGetLastError();
  }
  hipStreamSynchronize(p.stream);
  hipFree(h);
  return e;
}

hipError_t launch_mlp_forward(const float *params, const float *feat, int64_t M, float *c, hipStream_t s) {
  k_mlp_forward<<<nb(M), 256, 0, s>>>(params, feat, M, c);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *params, const float *feat, const float *dc, int64_t M, float *grad,
                               hipStream_t s) {
  const int nblocks = (int)((M + kBP - 1) / kBP);
  float *partial = nullptr;
  hipError_t e = hipMalloc(&partial, (size_t)nblocks * kNParams * sizeof(float));
  if (e != hipSuccess) return e;
  k_mlp_backward<<<nblocks, kBP, 0, s>>>(params, feat, dc, M, partial);
  k_reduce_partials<<<nb(kNParams), 256, 0, s>>>(partial, nblocks, grad);
  e = hipGetLastError();
  hipStreamSynchronize(s);
  hipFree(partial);
  return e;
}

// ---- backward without allocation (sgl_mlp_backward_noalloc)
// The per-block partial gradients live in this file-scope device array instead
// of a per-call allocation: kNoAllocBlocks blocks of kBP points, i.e. at most
// SGL_MLP_NOALLOC_MAX_POINTS points (46.5 MB per device, held until the
// process ends).  Each device holds its own copy at its own address; host code
// never passes the array's name (a host-side stand-in) to a kernel, only the
// address hipGetSymbolAddress returned for that device.
constexpr int kNoAllocBlocks = SGL_MLP_NOALLOC_MAX_POINTS / kBP;
static_assert(kNoAllocBlocks * kBP == SGL_MLP_NOALLOC_MAX_POINTS, "whole blocks");
static __device__ __align__(256) float scratch[(size_t)kNoAllocBlocks * kNParams];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device with
// that device current.
static hipError_t scratch_on(int device, float **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch[device] = (float *)ptr;
  }
  *out = g_scratch[device];
  return hipSuccess;
}

hipError_t launch_mlp_backward_noalloc(const float *params, const float *feat, const float *dc, int64_t M,
                                       float *grad, hipStream_t s, int device) {
  float *partial = nullptr;
  const hipError_t e = scratch_on(device, &partial);
  if (e != hipSuccess) return e;
  // the same kernels and summation order as launch_mlp_backward; every
  // partial the reduction reads is written first, so nothing is cleared
  const int nblocks = (int)((M + kBP - 1) / kBP);
  k_mlp_backward<<<nblocks, kBP, 0, s>>>(params, feat, dc, M, partial);
  k_reduce_partials<<<nb(kNParams), 256, 0, s>>>(partial, nblocks, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_adam<<<nb(n), 256, 0, s>>>(params, grad, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_weights(const Plan &p, const float *c, const float *feat, void *w) {
  const double rho2 = p.rho * p.rho;
  if (p.prec == SGL_F64)
    k_weights<double><<<nb(p.M), 256, 0, p.stream>>>(c, feat, p.M, rho2, (double *)w);
  else
    k_weights<float><<<nb(p.M), 256, 0, p.stream>>>(c, feat, p.M, rho2, (float *)w);
  return hipGetLastError();
}

hipError_t launch_weight_grad(const Plan &p, const void *y, const void *g, const void *w, double scale,
                              bool accumulate, float *dc) {
  if (p.prec == SGL_F64)
    k_weight_grad<double><<<nb(p.M), 256, 0, p.stream>>>((const cplx<double> *)y, (const cplx<double> *)g,
                                                         (const double *)w, p.M, scale, accumulate, dc);
  else
    k_weight_grad<float><<<nb(p.M), 256, 0, p.stream>>>((const cplx<float> *)y, (const cplx<float> *)g,
                                                        (const float *)w, p.M, scale, accumulate, dc);
  return hipGetLastError();
}

hipError_t launch_scale_by(const Plan &p, void *out, const void *a, const void *w, int64_t n) {
  if (p.prec == SGL_F64)
    k_scale_by<double><<<nb(n), 256, 0, p.stream>>>((cplx<double> *)out, (const cplx<double> *)a,
                                                    (const double *)w, n);
  else
    k_scale_by<float><<<nb(n), 256, 0, p.stream>>>((cplx<float> *)out, (const cplx<float> *)a, (const float *)w,
                                                   n);
  return hipGetLastError();
}

hipError_t launch_sub_from(const Plan &p, void *a, const void *b, int64_t n) {
  if (p.prec == SGL_F64)
    k_sub_from<double><<<nb(n), 256, 0, p.stream>>>((cplx<double> *)a, (const cplx<double> *)b, n);
  else
    k_sub_from<float><<<nb(n), 256, 0, p.stream>>>((cplx<float> *)a, (const cplx<float> *)b, n);
  return hipGetLastError();
}

hipError_t launch_norm2(const Plan &p, const void *a, int64_t n, double *out_dev) {
  if (p.prec == SGL_F64)
    k_norm2<double><<<1, 256, 0, p.stream>>>((const cplx<double> *)a, n, out_dev);
  else
    k_norm2<float><<<1, 256, 0, p.stream>>>((const cplx<float> *)a, n, out_dev);
  return hipGetLastError();
}

}  // namespace sgl
