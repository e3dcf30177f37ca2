/*
 * ORACLE — test infrastructure only.  Only tests/, the smoke entry point and
 * the CPU-baseline leg of bench.py may load this library.  The product path
 * (paper_1809_10786_amd) never calls it and shares no code with it.
 *
 * Exact non-lattice discrete SGL Fourier transform (NDSGLFT, Def. 1.3) and its
 * adjoint, by direct summation over all B(B+1)(2B+1)/6 basis functions at every
 * point:  f_i = sum_mu fhat_mu H_{n l m}(x_i)        (Def. 1.3, eq. (1.2))
 *         fhat_mu = sum_i conj(H_{n l m}(x_i)) y_i   (the Hermitian transpose)
 *
 * Basis (Def. 1.1): H_nlm = N_nl R_nl(r) Y_lm(theta, phi) with
 *   N_nl = sqrt(2 (n-l-1)! / Gamma(n+1/2)),   R_nl = L_{n-l-1}^{(l+1/2)}(r^2) r^l,
 *   Y_lm = Q_lm P_lm(cos theta) e^{i m phi},  Q_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
 * and P_lm the associated Legendre function in Rodrigues form carrying the
 * factor (-1)^m (Section 4).  Index order mu = n(n-1)(2n-1)/6 + l(l+1) + m
 * (Section 1).
 *
 * Evaluation per point, O(B^3) work:
 *  - radial: N_nl L_k^{(a)}(r^2), k = n-l-1, a = l+1/2, equals sqrt(2) p_k^{(a)}(r^2)
 *    with p_k the orthonormal Laguerre polynomial (since Gamma(k+a+1) = Gamma(n+1/2)),
 *    evaluated by the standard three-term recurrence of the Laguerre polynomials
 *    rescaled to orthonormal form; r^l/sqrt(Gamma(l+3/2)) is folded in through
 *    logarithms so that nothing overflows.
 *  - polar: Pbar_lm = Q_lm P_lm(cos theta) for 0 <= m <= l from the degree
 *    recurrence of Section 4 (eq. Legendre_recurrence) written for the
 *    normalised functions, seeded by the sectoral values Pbar_mm; negative m by
 *    Pbar_{l,-m} = (-1)^m Pbar_{l,m}.
 *  - azimuth: cos(m phi), sin(m phi) from libm.
 *
 * Parity status: pinned (closed forms for low n, orthonormality under a product
 * quadrature, scipy special functions, invariants, adjoint identity; see tests).
 *
 * Build: compiled twice, as double (default) and with -DORACLE_LONG_DOUBLE as
 * the 80-bit extended type the paper used for its radial recurrences
 * (Section 8); inputs/outputs are double in both builds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_LONG_DOUBLE
typedef long double real;
#define R_SQRT sqrtl
#define R_EXP expl
#define R_LOG logl
#define R_LGAMMA lgammal
#define R_COS cosl
#define R_SIN sinl
#define R_ATAN2 atan2l
#define R_HYPOT hypotl
#define R_PI 3.141592653589793238462643383279502884L
#define SYM(name) name##_ld
#else
typedef double real;
#define R_SQRT sqrt
#define R_EXP exp
#define R_LOG log
#define R_LGAMMA lgamma
#define R_COS cos
#define R_SIN sin
#define R_ATAN2 atan2
#define R_HYPOT hypot
#define R_PI 3.141592653589793238462643383279502884
#define SYM(name) name
#endif

int64_t SYM(oracle_num_coeffs)(int32_t B) {
  return (int64_t)B * (B + 1) * (2 * B + 1) / 6;
}

/* mu(n,l,m) of Section 1 (exact in integer arithmetic). */
int64_t SYM(oracle_mu)(int32_t n, int32_t l, int32_t m) {
  return (int64_t)n * (n - 1) * (2 * n - 1) / 6 + (int64_t)l * (l + 1) + m;
}

/* Radial table: rad[l*B + (n-1)] = N_nl R_nl(r) for 0 <= l < n <= B. */
static void radial_table(int32_t B, real r, real *rad) {
  const real x = r * r;
  for (int32_t l = 0; l < B; ++l) {
    const real a = (real)l + (real)0.5;
    /* sqrt(2) r^l / sqrt(Gamma(l + 3/2)) = sqrt(2) r^l p_0^{(a)}.              */
    real seed;
    if (r == 0) {
      seed = (l == 0) ? R_SQRT((real)2) * R_EXP(-(real)0.5 * R_LGAMMA((real)1.5)) : 0;
    } else {
      seed = R_EXP((real)l * R_LOG(r) - (real)0.5 * R_LGAMMA(a + 1) + (real)0.5 * R_LOG((real)2));
    }
    real pkm1 = 0, pk = seed;
    for (int32_t n = l + 1; n <= B; ++n) {
      const int32_t k = n - l - 1;
      rad[l * B + (n - 1)] = pk;
      /* p_{k+1} = ((2k+a+1-x) p_k - sqrt(k(k+a)) p_{k-1}) / sqrt((k+1)(k+a+1)) */
      const real pkp1 = ((2 * (real)k + a + 1 - x) * pk - R_SQRT((real)k * ((real)k + a)) * pkm1) /
                        R_SQRT(((real)k + 1) * ((real)k + a + 1));
      pkm1 = pk;
      pk = pkp1;
    }
  }
}

/* Polar table: leg[l*B + m] = Q_lm P_lm(ct) for 0 <= m <= l < B (Condon-Shortley sign). */
static void legendre_table(int32_t B, real ct, real st, real *leg) {
  real pmm = R_SQRT((real)1 / (4 * R_PI));
  for (int32_t m = 0; m < B; ++m) {
    if (m > 0) pmm = -R_SQRT((2 * (real)m + 1) / (2 * (real)m)) * st * pmm;
    leg[m * B + m] = pmm;
    if (m + 1 < B) leg[(m + 1) * B + m] = R_SQRT(2 * (real)m + 3) * ct * pmm;
    for (int32_t l = m + 2; l < B; ++l) {
      const real a = R_SQRT((4 * (real)l * l - 1) / ((real)l * l - (real)m * m));
      const real b = R_SQRT((((real)l - 1) * ((real)l - 1) - (real)m * m) /
                            (4 * ((real)l - 1) * ((real)l - 1) - 1));
      leg[l * B + m] = a * (ct * leg[(l - 1) * B + m] - b * leg[(l - 2) * B + m]);
    }
  }
}

/* Spherical coordinates (Section 1); theta, phi are arbitrary but fixed at the
 * origin / on the z axis, where every surviving term does not depend on them. */
static void spherical(const double *p, real *r, real *ct, real *st, real *phi) {
  const real x = p[0], y = p[1], z = p[2];
  const real rxy = R_HYPOT(x, y);
  *r = R_HYPOT(rxy, z);
  const real th = R_ATAN2(rxy, z);
  *ct = R_COS(th);
  *st = R_SIN(th);
  real ph = R_ATAN2(y, x);
  if (ph < 0) ph += 2 * R_PI;
  *phi = ph;
}

/* All Nc basis values H_mu(x) at one point (interleaved re, im). */
void SYM(oracle_basis)(int32_t B, const double *point, double *h_out) {
  real *rad = (real *)malloc(sizeof(real) * B * B);
  real *leg = (real *)malloc(sizeof(real) * B * B);
  real r, ct, st, phi;
  spherical(point, &r, &ct, &st, &phi);
  radial_table(B, r, rad);
  legendre_table(B, ct, st, leg);
  for (int32_t n = 1; n <= B; ++n)
    for (int32_t l = 0; l < n; ++l)
      for (int32_t m = -l; m <= l; ++m) {
        const int32_t am = m < 0 ? -m : m;
        real p = leg[l * B + am];
        if (m < 0 && (am & 1)) p = -p;
        const real v = rad[l * B + (n - 1)] * p;
        const int64_t mu = SYM(oracle_mu)(n, l, m);
        h_out[2 * mu] = (double)(v * R_COS((real)m * phi));
        h_out[2 * mu + 1] = (double)(v * R_SIN((real)m * phi));
      }
  free(rad);
  free(leg);
}

/* f = Lambda fhat.  points: M x 3 (x,y,z); fhat: Nc complex; f: M complex. */
int SYM(oracle_forward)(int32_t B, int64_t M, const double *points, const double *fhat, double *f,
                        int32_t nthreads) {
  if (B < 1 || M < 0) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    real *rad = (real *)malloc(sizeof(real) * B * B);
    real *leg = (real *)malloc(sizeof(real) * B * B);
    real *cm = (real *)malloc(sizeof(real) * (2 * B));
    real *sm = (real *)malloc(sizeof(real) * (2 * B));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
      real r, ct, st, phi;
      spherical(points + 3 * i, &r, &ct, &st, &phi);
      radial_table(B, r, rad);
      legendre_table(B, ct, st, leg);
      for (int32_t m = 0; m < B; ++m) {
        cm[m] = R_COS((real)m * phi);
        sm[m] = R_SIN((real)m * phi);
      }
      real acc_re = 0, acc_im = 0;
      for (int32_t l = 0; l < B; ++l)
        for (int32_t m = -l; m <= l; ++m) {
          /* g_lm(r) = sum_n fhat_nlm N_nl R_nl(r)  (Section 6) */
          real g_re = 0, g_im = 0;
          for (int32_t n = l + 1; n <= B; ++n) {
            const int64_t mu = SYM(oracle_mu)(n, l, m);
            const real w = rad[l * B + (n - 1)];
            g_re += w * (real)fhat[2 * mu];
            g_im += w * (real)fhat[2 * mu + 1];
          }
          const int32_t am = m < 0 ? -m : m;
          real p = leg[l * B + am];
          if (m < 0 && (am & 1)) p = -p;
          const real c = cm[am], s = (m < 0) ? -sm[am] : sm[am];
          /* += g * p * e^{i m phi} */
          acc_re += p * (g_re * c - g_im * s);
          acc_im += p * (g_re * s + g_im * c);
        }
      f[2 * i] = (double)acc_re;
      f[2 * i + 1] = (double)acc_im;
    }
    free(rad);
    free(leg);
    free(cm);
    free(sm);
  }
  return 0;
}

/* fhat = Lambda^H y.  Per-thread accumulators, summed in thread order. */
int SYM(oracle_adjoint)(int32_t B, int64_t M, const double *points, const double *y, double *fhat,
                        int32_t nthreads) {
  if (B < 1 || M < 0) return -1;
  const int64_t nc = SYM(oracle_num_coeffs)(B);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const int nt = omp_get_max_threads();
#else
  (void)nthreads;
  const int nt = 1;
#endif
  real *acc = (real *)calloc((size_t)nt * 2 * nc, sizeof(real));
  if (!acc) return -3;
#pragma omp parallel
  {
#ifdef _OPENMP
    const int tid = omp_get_thread_num();
#else
    const int tid = 0;
#endif
    real *mine = acc + (size_t)tid * 2 * nc;
    real *rad = (real *)malloc(sizeof(real) * B * B);
    real *leg = (real *)malloc(sizeof(real) * B * B);
    real *cm = (real *)malloc(sizeof(real) * (2 * B));
    real *sm = (real *)malloc(sizeof(real) * (2 * B));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
      real r, ct, st, phi;
      spherical(points + 3 * i, &r, &ct, &st, &phi);
      radial_table(B, r, rad);
      legendre_table(B, ct, st, leg);
      for (int32_t m = 0; m < B; ++m) {
        cm[m] = R_COS((real)m * phi);
        sm[m] = R_SIN((real)m * phi);
      }
      const real y_re = (real)y[2 * i], y_im = (real)y[2 * i + 1];
      for (int32_t l = 0; l < B; ++l)
        for (int32_t m = -l; m <= l; ++m) {
          const int32_t am = m < 0 ? -m : m;
          real p = leg[l * B + am];
          if (m < 0 && (am & 1)) p = -p;
          const real c = cm[am], s = (m < 0) ? -sm[am] : sm[am];
          /* t = conj(p e^{i m phi}) y */
          const real t_re = p * (c * y_re + s * y_im);
          const real t_im = p * (c * y_im - s * y_re);
          for (int32_t n = l + 1; n <= B; ++n) {
            const int64_t mu = SYM(oracle_mu)(n, l, m);
            const real w = rad[l * B + (n - 1)];
            mine[2 * mu] += w * t_re;
            mine[2 * mu + 1] += w * t_im;
          }
        }
    }
    free(rad);
    free(leg);
    free(cm);
    free(sm);
  }
  for (int64_t k = 0; k < 2 * nc; ++k) {
    real s = 0;
    for (int t = 0; t < nt; ++t) s += acc[(size_t)t * 2 * nc + k];
    fhat[k] = (double)s;
  }
  free(acc);
  return 0;
}

int SYM(oracle_max_threads)(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
