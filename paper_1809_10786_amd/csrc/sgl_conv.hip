// Conversion between SGL coefficients fhat (order mu, Section 1) and the
// trigonometric coefficients eta of eq. nfsglft_nfft on the 4B x 2B x 2B grid
// (Remark 8.1): the factors of Thm. 6.2 to the right of N, as two batched
// dense products with the collapsed tables built on the host:
//
//   radial  (per l):  beta_m[l][a]  = sum_k K_l[a][k] fhat(n = l+1+k, l, m),  a = |kappa0|
//   polar   (per m):  zeta_m[k1][a] = sum_l Kp_m[k1][l] beta_m[l][a]
//   eta[+-a][+-k1][m] = zeta_m[|k1|][a]            (even m)
//                     = -i sgn(k1) S_m[|k1|] beta  (odd m)
//
// and the exact adjoints of both (Cor. 6.3).  eta index:
// ((k0 + 2B) * 2B + (k1 + B)) * 2B + (m + B).
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
__device__ inline int64_t eta_index(int B, int k0, int k1, int m) {
  return ((int64_t)(k0 + 2 * B) * (2 * B) + (k1 + B)) * (2 * B) + (m + B);
}

// beta_m[l][a] = sum_k K_l[a][k] fhat(l+1+k, l, m);  thread per (m, l, a).
template <class R>
__global__ __launch_bounds__(256) void k_radial(int B, const R *__restrict__ krad, const cplx<R> *__restrict__ fhat,
                                                cplx<R> *__restrict__ beta) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)A * B * A) return;
  const int a = (int)(t % A);
  const int l = (int)((t / A) % B);
  const int m = (int)(t / ((int64_t)A * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  if (l < am) return;
  const int K = B - l;
  const R *row = krad + krad_offset(B, l) + (int64_t)a * K;
  R sr = 0, si = 0;
  for (int k = 0; k < K; ++k) {
    const cplx<R> v = fhat[mu_index(l + 1 + k, l, m)];
    sr += row[k] * v.re;
    si += row[k] * v.im;
  }
  beta[beta_offset(B, m) + (int64_t)(l - am) * A + a] = {sr, si};
}

// Polar product and unfolding into every eta entry; thread per
// (m + B in [0, 2B), k1 in [0, B], a in [0, 2B]); entries outside the support
// (m = -B, k1 = -B, |k0| >= 2B-1) are written as zero.
template <class R>
__global__ __launch_bounds__(256) void k_polar(int B, const R *__restrict__ kpol, const cplx<R> *__restrict__ beta,
                                               cplx<R> *__restrict__ eta) {
  const int NA = 2 * B + 1, NK = B + 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)NA * NK * 2 * B) return;
  const int a = (int)(t % NA);
  const int k1 = (int)((t / NA) % NK);
  const int m = (int)(t / ((int64_t)NA * NK)) - B;
  const int am = m < 0 ? -m : m;
  cplx<R> v = {0, 0};
  if (m > -B && k1 < B && a < 2 * B - 1) {
    const int K = B - am;
    const R *row = kpol + kpol_offset(B, am) + (int64_t)k1 * K;
    const cplx<R> *col = beta + beta_offset(B, m) + a;
    R sr = 0, si = 0;
    for (int c = 0; c < K; ++c) {
      const cplx<R> b = col[(int64_t)c * (2 * B - 1)];
      sr += row[c] * b.re;
      si += row[c] * b.im;
    }
    if (m < 0 && (am & 1)) {  // Kp_{-m} = (-1)^m Kp_m
      sr = -sr;
      si = -si;
    }
    if (am & 1) v = {si, -sr};  // -i * s
    else v = {sr, si};
  }
  const bool odd = (am & 1) != 0;
  for (int s0 = 0; s0 < 2; ++s0) {
    const int k0 = s0 ? -a : a;
    if (k0 >= 2 * B || (s0 && a == 0)) continue;
    for (int s1 = 0; s1 < 2; ++s1) {
      const int kk1 = s1 ? -k1 : k1;
      if (kk1 >= B || (s1 && k1 == 0)) continue;
      cplx<R> w = v;
      if (odd && s1) w = {-v.re, -v.im};
      eta[eta_index(B, k0, kk1, m)] = w;
    }
  }
}

// Adjoint of k_polar: betaH_m[l][a] = sum_k1 Kp_m[k1][l]^* zetaH_m[k1][a], with
// zetaH gathered from the mirrored eta entries.  Thread per (m, l, a).
template <class R>
__global__ __launch_bounds__(256) void k_polar_adj(int B, const R *__restrict__ kpol, const cplx<R> *__restrict__ eta,
                                                   cplx<R> *__restrict__ beta) {
  const int A = 2 * B - 1;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)A * B * A) return;
  const int a = (int)(t % A);
  const int l = (int)((t / A) % B);
  const int m = (int)(t / ((int64_t)A * B)) - (B - 1);
  const int am = m < 0 ? -m : m;
  if (l < am) return;
  const int K = B - am;
  const R *tab = kpol + kpol_offset(B, am) + (l - am);
  const bool odd = (am & 1) != 0;
  R sr = 0, si = 0;
  for (int k1 = odd ? 1 : 0; k1 < B; ++k1) {
    R zr = 0, zi = 0;
    for (int s0 = 0; s0 < 2; ++s0) {
      if (s0 && a == 0) continue;
      const int k0 = s0 ? -a : a;
      const cplx<R> p = eta[eta_index(B, k0, k1, m)];
      zr += p.re;
      zi += p.im;
      if (k1 > 0) {
        const cplx<R> n = eta[eta_index(B, k0, -k1, m)];
        if (odd) {
          zr -= n.re;
          zi -= n.im;
        } else {
          zr += n.re;
          zi += n.im;
        }
      }
    }
    const R kv = tab[(int64_t)k1 * K];
    sr += kv * zr;
    si += kv * zi;
  }
  if (m < 0 && odd) {
    sr = -sr;
    si = -si;
  }
  cplx<R> out;
  if (odd) out = {-si, sr};  // (-i)^* = +i
  else out = {sr, si};
  beta[beta_offset(B, m) + (int64_t)(l - am) * A + a] = out;
}

// Adjoint of k_radial: fhat(l+1+k, l, m) = sum_a K_l[a][k] betaH_m[l][a].
template <class R>
__global__ __launch_bounds__(256) void k_radial_adj(int B, const R *__restrict__ krad, const cplx<R> *__restrict__ beta,
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
  const R *col = krad + krad_offset(B, l) + k;
  const cplx<R> *bl = beta + beta_offset(B, m) + (int64_t)(l - am) * A;
  R sr = 0, si = 0;
  for (int a = 0; a < A; ++a) {
    const R kv = col[(int64_t)a * K];
    sr += kv * bl[a].re;
    si += kv * bl[a].im;
  }
  fhat[mu_index(l + 1 + k, l, m)] = {sr, si};
}

template <class R>
hipError_t radial(const Plan &p, const void *fhat) {
  const int B = p.B, A = 2 * B - 1;
  const int64_t n = (int64_t)A * B * A;
  k_radial<R><<<(int)((n + 255) / 256), 256, 0, p.stream>>>(B, (const R *)p.krad, (const cplx<R> *)fhat,
                                                            (cplx<R> *)p.beta);
  return hipGetLastError();
}

template <class R>
hipError_t polar(const Plan &p, void *eta) {
  const int B = p.B;
  const int64_t n = (int64_t)(2 * B + 1) * (B + 1) * 2 * B;
  k_polar<R><<<(int)((n + 255) / 256), 256, 0, p.stream>>>(B, (const R *)p.kpol, (const cplx<R> *)p.beta,
                                                           (cplx<R> *)eta);
  return hipGetLastError();
}

template <class R>
hipError_t polar_adj(const Plan &p, const void *eta) {
  const int B = p.B, A = 2 * B - 1;
  const int64_t n = (int64_t)A * B * A;
  k_polar_adj<R><<<(int)((n + 255) / 256), 256, 0, p.stream>>>(B, (const R *)p.kpol, (const cplx<R> *)eta,
                                                               (cplx<R> *)p.beta);
  return hipGetLastError();
}

template <class R>
hipError_t radial_adj(const Plan &p, void *fhat) {
  const int B = p.B, A = 2 * B - 1;
  const int64_t n = (int64_t)B * B * A;
  k_radial_adj<R><<<(int)((n + 255) / 256), 256, 0, p.stream>>>(B, (const R *)p.krad, (const cplx<R> *)p.beta,
                                                                (cplx<R> *)fhat);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_conv_radial(const Plan &p, const void *fhat) {
  return p.prec == SGL_F64 ? radial<double>(p, fhat) : radial<float>(p, fhat);
}
hipError_t launch_conv_polar(const Plan &p, void *eta) {
  return p.prec == SGL_F64 ? polar<double>(p, eta) : polar<float>(p, eta);
}
hipError_t launch_conv_polar_adj(const Plan &p, const void *eta) {
  return p.prec == SGL_F64 ? polar_adj<double>(p, eta) : polar_adj<float>(p, eta);
}
hipError_t launch_conv_radial_adj(const Plan &p, void *fhat) {
  return p.prec == SGL_F64 ? radial_adj<double>(p, fhat) : radial_adj<float>(p, fhat);
}

}  // namespace sgl
