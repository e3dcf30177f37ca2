// Conversion between SGL coefficients fhat (order mu, Section 1) and the
// trigonometric coefficients eta of eq. nfsglft_nfft on the 4B x 2B x 2B grid
// (Remark 8.1): the factors of Thm. 6.2 to the right of N, as two batched
// dense products with the collapsed tables built on the host:
//
//   radial  (per l):  beta_m[l][a]  = sum_k K_l[a][k] fhat(n = l+1+k, l, m),  a = |kappa0|
//   polar   (per m):  zeta_m[k1][a] = sum_l Kp_m[k1][l] beta_m[l][a],          k1 >= 0
//   unfold:           eta[+-a][+-k1][m] = zeta_m[k1][a]                (even m)
//                     eta[+-a][ +-k1][m] = +- (-i) zeta_m[k1][a]       (odd m)
//
// and the exact adjoints of all three (Cor. 6.3).  The products always run in
// FP64 with FP64 tables: the tables carry the growth of the radial functions
// towards r = rho, and their sums cancel strongly, so the FP32 mode keeps only
// its inputs and outputs in FP32.
// eta index: ((k0 + 2B) * 2B + (k1 + B)) * 2B + (m + B).
// zeta (compact) index: (m + B - 1) * B * (2B - 1) + k1 * (2B - 1) + a.
#include "sgl_internal.h"

namespace sgl {

namespace {

__device__ inline int64_t mu_index(int n, int l, int m) {
  return (int64_t)n * (n - 1) * (2 * n - 1) / 6 + (int64_t)l * (l + 1) + m;
}
// K_l starts at (2B-1) * sum_{l' < l} (B - l').
__device__ inline int64_t krad_offset(int B, int l) {
  return (int64_t)(2 * B - 1) * ((int64_t)l * B - (int64_t)l * (l - 1) / 2);
}
// Kp_m (m >= 0) starts at B * sum_{m' < m} (B - m').
__device__ inline int64_t kpol_offset(int B, int m) {
  return (int64_t)B * ((int64_t)m * B - (int64_t)m * (m - 1) / 2);
}
// beta_m block (rows l = |m|..B-1, columns a = 0..2B-2) starts at
// (2B-1) * sum_{m' = 1-B}^{m-1} (B - |m'|).
__device__ inline int64_t beta_offset(int B, int m) {
  int64_t c;
  if (m <= 0) c = (int64_t)(B + m - 1) * (B + m) / 2;
  else c = (int64_t)B * (B - 1) / 2 + (int64_t)m * B - (int64_t)m * (m - 1) / 2;
  return c * (2 * B - 1);
}
__device__ inline int64_t zeta_index(int B, int m, int k1, int a) {
  return ((int64_t)(m + B - 1) * B + k1) * (2 * B - 1) + a;
}
__device__ inline int64_t eta_index(int B, int k0, int k1, int m) {
  return ((int64_t)(k0 + 2 * B) * (2 * B) + (k1 + B)) * (2 * B) + (m + B);
}

// beta_m[l][a] = sum_k K_l[a][k] fhat(l+1+k, l, m);  thread per (m, l, a), a fastest.
template <class R>
__global__ __launch_bounds__(256) void k_radial(int B, const double *__restrict__ krad,
                                                const cplx<R> *__restrict__ fhat, cplx<double> *__restrict__ beta) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)A * B * A) return;
  const int a = (int)(t % A);
  const int l = (int)((t / A) % B);
  const int m = (int)(t / ((int64_t)A * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  if (l < am) return;
  const int K = B - l;
  const double *row = krad + krad_offset(B, l) + (int64_t)a * K;
  double sr = 0, si = 0;
  for (int k = 0; k < K; ++k) {
    const cplx<R> v = fhat[mu_index(l + 1 + k, l, m)];
    sr += row[k] * (double)v.re;
    si += row[k] * (double)v.im;
  }
  beta[beta_offset(B, m) + (int64_t)(l - am) * A + a] = {sr, si};
}

// zeta_m[k1][a] = sum_l Kp_m[k1][l] beta_m[l][a], with Kp_{-m} = (-1)^m Kp_m;
// thread per (m, k1, a), a fastest.
__global__ __launch_bounds__(256) void k_polar(int B, const double *__restrict__ kpol,
                                               const cplx<double> *__restrict__ beta,
                                               cplx<double> *__restrict__ zeta) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)A * B * A) return;
  const int a = (int)(t % A);
  const int k1 = (int)((t / A) % B);
  const int m = (int)(t / ((int64_t)A * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  const int K = B - am;
  const double *row = kpol + kpol_offset(B, am) + (int64_t)k1 * K;
  const cplx<double> *col = beta + beta_offset(B, m) + a;
  double sr = 0, si = 0;
  for (int c = 0; c < K; ++c) {
    const cplx<double> b = col[(int64_t)c * A];
    sr += row[c] * b.re;
    si += row[c] * b.im;
  }
  if (m < 0 && (am & 1)) {
    sr = -sr;
    si = -si;
  }
  zeta[zeta_index(B, m, k1, a)] = {sr, si};
}

// Every eta entry from the compact zeta; entries outside the support
// (m = -B, k1 = -B, |k0| >= 2B-1) are zero.  Thread per eta entry, m fastest.
template <class R>
__global__ __launch_bounds__(256) void k_unfold(int B, const cplx<double> *__restrict__ zeta,
                                                cplx<R> *__restrict__ eta) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)4 * B * 2 * B * 2 * B) return;
  const int m = (int)(t % (2 * B)) - B;
  const int k1 = (int)((t / (2 * B)) % (2 * B)) - B;
  const int k0 = (int)(t / ((int64_t)4 * B * B)) - 2 * B;
  const int a = k0 < 0 ? -k0 : k0, ak1 = k1 < 0 ? -k1 : k1, am = m < 0 ? -m : m;
  cplx<R> v = {0, 0};
  if (m > -B && k1 > -B && a < 2 * B - 1) {
    const cplx<double> z = zeta[zeta_index(B, m, ak1, a)];
    if (am & 1) {
      // -i sgn(k1) z
      const double s = k1 > 0 ? 1.0 : (k1 < 0 ? -1.0 : 0.0);
      v = {(R)(s * z.im), (R)(-s * z.re)};
    } else {
      v = {(R)z.re, (R)z.im};
    }
  }
  eta[t] = v;
}

// Adjoint of k_unfold: zetaH_m[k1][a] = sum over the mirrored entries, with the
// conjugate factor (+i sgn(k1)) for odd m.  Thread per (m, k1, a), a fastest.
template <class R>
__global__ __launch_bounds__(256) void k_fold_eta(int B, const cplx<R> *__restrict__ eta,
                                                  cplx<double> *__restrict__ zeta) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)A * B * A) return;
  const int a = (int)(t % A);
  const int k1 = (int)((t / A) % B);
  const int m = (int)(t / ((int64_t)A * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  const bool odd = (am & 1) != 0;
  double zr = 0, zi = 0;
  for (int s0 = 0; s0 < 2; ++s0) {
    if (s0 && a == 0) continue;
    const int k0 = s0 ? -a : a;
    for (int s1 = 0; s1 < 2; ++s1) {
      if (s1 && k1 == 0) continue;
      const int kk1 = s1 ? -k1 : k1;
      const cplx<R> e = eta[eta_index(B, k0, kk1, m)];
      if (odd) {
        // conj(-i sgn) = +i sgn: (+i)(x + iy) = -y + ix
        const double s = kk1 > 0 ? 1.0 : (kk1 < 0 ? -1.0 : 0.0);
        zr += -s * (double)e.im;
        zi += s * (double)e.re;
      } else {
        zr += (double)e.re;
        zi += (double)e.im;
      }
    }
  }
  zeta[zeta_index(B, m, k1, a)] = {zr, zi};
}

// betaH_m[l][a] = sum_k1 Kp_m[k1][l] zetaH_m[k1][a];  thread per (m, l, a).
__global__ __launch_bounds__(256) void k_polar_adj(int B, const double *__restrict__ kpol,
                                                   const cplx<double> *__restrict__ zeta,
                                                   cplx<double> *__restrict__ beta) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)A * B * A) return;
  const int a = (int)(t % A);
  const int l = (int)((t / A) % B);
  const int m = (int)(t / ((int64_t)A * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  if (l < am) return;
  const int K = B - am;
  const double *tab = kpol + kpol_offset(B, am) + (l - am);
  const cplx<double> *z = zeta + zeta_index(B, m, 0, a);
  double sr = 0, si = 0;
  for (int k1 = 0; k1 < B; ++k1) {
    const double kv = tab[(int64_t)k1 * K];
    const cplx<double> v = z[(int64_t)k1 * A];
    sr += kv * v.re;
    si += kv * v.im;
  }
  if (m < 0 && (am & 1)) {
    sr = -sr;
    si = -si;
  }
  beta[beta_offset(B, m) + (int64_t)(l - am) * A + a] = {sr, si};
}

// fhat(l+1+k, l, m) = sum_a K_l[a][k] betaH_m[l][a];  thread per (m, l, k).
template <class R>
__global__ __launch_bounds__(256) void k_radial_adj(int B, const double *__restrict__ krad,
                                                    const cplx<double> *__restrict__ beta,
                                                    cplx<R> *__restrict__ fhat) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * B * A) return;
  const int k = (int)(t % B);
  const int l = (int)((t / B) % B);
  const int m = (int)(t / ((int64_t)B * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  if (l < am || k >= B - l) return;
  const int K = B - l;
  const double *col = krad + krad_offset(B, l) + k;
  const cplx<double> *bl = beta + beta_offset(B, m) + (int64_t)(l - am) * A;
  double sr = 0, si = 0;
  for (int a = 0; a < A; ++a) {
    const double kv = col[(int64_t)a * K];
    sr += kv * bl[a].re;
    si += kv * bl[a].im;
  }
  fhat[mu_index(l + 1 + k, l, m)] = {(R)sr, (R)si};
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class R>
hipError_t radial(const Plan &p, const void *fhat) {
  const int B = p.B, A = 2 * B - 1;
  k_radial<R><<<nblk((int64_t)A * B * A), 256, 0, p.stream>>>(B, (const double *)p.krad, (const cplx<R> *)fhat,
                                                              (cplx<double> *)p.beta);
  return hipGetLastError();
}

template <class R>
hipError_t polar(const Plan &p, void *eta) {
  const int B = p.B, A = 2 * B - 1;
  k_polar<<<nblk((int64_t)A * B * A), 256, 0, p.stream>>>(B, (const double *)p.kpol, (const cplx<double> *)p.beta,
                                                          (cplx<double> *)p.zeta);
  k_unfold<R><<<nblk((int64_t)16 * B * B * B), 256, 0, p.stream>>>(B, (const cplx<double> *)p.zeta,
                                                                   (cplx<R> *)eta);
  return hipGetLastError();
}

template <class R>
hipError_t polar_adj(const Plan &p, const void *eta) {  // R: element type of eta
  const int B = p.B, A = 2 * B - 1;
  k_fold_eta<R><<<nblk((int64_t)A * B * A), 256, 0, p.stream>>>(B, (const cplx<R> *)eta, (cplx<double> *)p.zeta);
  k_polar_adj<<<nblk((int64_t)A * B * A), 256, 0, p.stream>>>(B, (const double *)p.kpol,
                                                              (const cplx<double> *)p.zeta, (cplx<double> *)p.beta);
  return hipGetLastError();
}

template <class R>
hipError_t radial_adj(const Plan &p, void *fhat) {
  const int B = p.B, A = 2 * B - 1;
  k_radial_adj<R><<<nblk((int64_t)B * B * A), 256, 0, p.stream>>>(B, (const double *)p.krad,
                                                                  (const cplx<double> *)p.beta, (cplx<R> *)fhat);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_conv_radial(const Plan &p, const void *fhat) {
  return p.prec == SGL_F64 ? radial<double>(p, fhat) : radial<float>(p, fhat);
}
hipError_t launch_conv_polar(const Plan &p, void *eta, int eta_f64) {
  return eta_f64 ? polar<double>(p, eta) : polar<float>(p, eta);
}
hipError_t launch_conv_polar_adj(const Plan &p, const void *eta, int eta_f64) {
  return eta_f64 ? polar_adj<double>(p, eta) : polar_adj<float>(p, eta);
}
hipError_t launch_conv_radial_adj(const Plan &p, void *fhat) {
  return p.prec == SGL_F64 ? radial_adj<double>(p, fhat) : radial_adj<float>(p, fhat);
}

}  // namespace sgl
