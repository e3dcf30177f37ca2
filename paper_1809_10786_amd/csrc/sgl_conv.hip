// Unfolding of the compact polar output zeta into the trigonometric
// coefficients eta of eq. nfsglft_nfft on the 4B x 2B x 2B grid (Remark 8.1),
// and its adjoint:
//
//   unfold:  eta[+-a][+-k1][m] = zeta_m[k1][a]                (even m)
//            eta[+-a][ +-k1][m] = +- (-i) zeta_m[k1][a]       (odd m)
//
// (the sign symmetries of Thm. 6.2 and Cor. 6.3).  The radial and polar
// products that produce and consume zeta are in sgl_conv_products.hip.
// eta index: ((k0 + 2B) * 2B + (k1 + B)) * 2B + (m + B).
// zeta (compact) index: (m + B - 1) * B * (2B - 1) + k1 * (2B - 1) + a.
#include "sgl_internal.h"

namespace sgl {

namespace {

__device__ inline int64_t zeta_index(int B, int m, int k1, int a) {
  return ((int64_t)(m + B - 1) * B + k1) * (2 * B - 1) + a;
}
__device__ inline int64_t eta_index(int B, int k0, int k1, int m) {
  return ((int64_t)(k0 + 2 * B) * (2 * B) + (k1 + B)) * (2 * B) + (m + B);
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

}  // namespace

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class R>
hipError_t unfold_only(const Plan &p, void *eta) {
  const int B = p.B;
  k_unfold<R><<<nblk((int64_t)16 * B * B * B), 256, 0, p.stream>>>(B, (const cplx<double> *)p.zeta, (cplx<R> *)eta);
  return hipGetLastError();
}
template <class R>
hipError_t fold_eta_only(const Plan &p, const void *eta) {
  const int B = p.B, A = 2 * B - 1;
  k_fold_eta<R><<<nblk((int64_t)A * B * A), 256, 0, p.stream>>>(B, (const cplx<R> *)eta, (cplx<double> *)p.zeta);
  return hipGetLastError();
}
hipError_t launch_conv_unfold(const Plan &p, void *eta, int eta_f64) {
  return eta_f64 ? unfold_only<double>(p, eta) : unfold_only<float>(p, eta);
}
hipError_t launch_conv_fold_eta(const Plan &p, const void *eta, int eta_f64) {
  return eta_f64 ? fold_eta_only<double>(p, eta) : fold_eta_only<float>(p, eta);
}

}  // namespace sgl
