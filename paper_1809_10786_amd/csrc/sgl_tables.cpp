// Host-side tables of the conversion (Section 6, Thm. 6.2), built in 80-bit
// long double -- the precision the paper used for its radial recurrences
// (Section 8) -- then rounded to the device precision.
//
// The fast algorithm multiplies, per l and per m, a small dense matrix into the
// coefficients.  Here every chain of fixed factors is collapsed into one matrix:
//
//  radial, per l (rows a = |kappa0| = 0..2B-2, columns k = n-l-1 = 0..B-l-1):
//     K_l[a][k] = (1/2B) sum_j cos(a w_j) N_nl R_nl(rho (1 + cos w_j) / 2),
//  which is the kappa0 >= 0 half of A_B D_2B C~_2B R_l (eqs. nfsglft_a_alpha,
//  nfsglft_a_beta): D_2B C~_2B = diag(1/2B, 2/2B, ...) C_2B and A_B halves
//  every coefficient but the first, so both cases give 1/2B; beta_{-a} = beta_a.
//
//  polar, per m >= 0 (rows k1 = 0..B-1, columns l = m..B-1):
//     even m:  K_m[k1][l] = (1/2B) sum_j cos(k1 w_j) Qbar P_lm(cos w_j)
//     odd m :  S_m[k1][l] = (1/2B) sum_j sin(k1 w_j) Qbar P_lm(cos w_j),
//  with zeta_{k1} = K_m[|k1|] beta (even m, eq. nfsglft_a_zeta_even) and
//  zeta_{k1} = -i S_m[k1] beta, S odd in k1 (odd m).  The odd-m form follows
//  from W_m D_2B C~_2B V_B (eqs. nfsglft_a_epsilon_odd, nfsglft_a_zeta_odd):
//  eps_{k-1} - eps_{k+1} = (1/B) sum_j [cos((k-1)w_j) - cos((k+1)w_j)] h_j / sin w_j
//  = (2/B) sum_j sin(k w_j) h_j, so the 1/sin w_j weighting cancels exactly
//  and no node ever divides by sin w_j.  Negative m use P_{l,-m} = (-1)^m ... so
//  that the normalised functions satisfy K_{-m} = (-1)^m K_m.
//
// The nodes are w_j = (2j+1) pi / (4B), j = 0..2B-1 (Section 6).
#include <cmath>
#include <vector>

#include "sgl_internal.h"

namespace sgl {

namespace {
constexpr long double kPi = 3.141592653589793238462643383279502884L;

long double node(int B, int j) { return (2.0L * j + 1.0L) * kPi / (4.0L * B); }
}  // namespace

// Generalised Laguerre polynomials L_k^{(alpha)}(x), k = 0..K-1, by the
// classical recurrence (k+1) L_{k+1} = (2k + alpha + 1 - x) L_k - (k + alpha) L_{k-1}.
static void laguerre(int K, long double alpha, long double x, long double *out) {
  long double lm1 = 0.0L, l0 = 1.0L;
  for (int k = 0; k < K; ++k) {
    out[k] = l0;
    const long double l1 = ((2.0L * k + alpha + 1.0L - x) * l0 - (k + alpha) * lm1) / (k + 1.0L);
    lm1 = l0;
    l0 = l1;
  }
}

void build_radial_table(int B, double rho, std::vector<long double> &out, std::vector<int64_t> &off) {
  off.assign(B + 1, 0);
  for (int l = 0; l < B; ++l) off[l + 1] = off[l] + (int64_t)(2 * B - 1) * (B - l);
  out.assign(off[B], 0.0L);
  std::vector<long double> lag(B);
  std::vector<long double> rad((size_t)2 * B * B);  // rad[j][k] for the current l
  std::vector<long double> ctab((size_t)4 * B * B);  // cos(a w_j)
  for (int a = 0; a < 2 * B; ++a)
    for (int j = 0; j < 2 * B; ++j) ctab[(size_t)a * 2 * B + j] = cosl(a * node(B, j));
  for (int l = 0; l < B; ++l) {
    const int K = B - l;
    const long double alpha = l + 0.5L;
    // N_nl = sqrt(2 (n-l-1)! / Gamma(n + 1/2))   (Def. 1.1), n = l + 1 + k
    std::vector<long double> Nn(K);
    for (int k = 0; k < K; ++k) Nn[k] = sqrtl(2.0L * expl(lgammal(k + 1.0L) - lgammal(l + 1 + k + 0.5L)));
    for (int j = 0; j < 2 * B; ++j) {
      const long double r = (long double)rho * (1.0L + cosl(node(B, j))) / 2.0L;
      laguerre(K, alpha, r * r, lag.data());
      const long double rl = powl(r, (long double)l);
      for (int k = 0; k < K; ++k) {
        rad[(size_t)j * K + k] = Nn[k] * lag[k] * rl;
      }
    }
    long double *Kl = out.data() + off[l];
    for (int a = 0; a < 2 * B - 1; ++a)
      for (int k = 0; k < K; ++k) {
        long double s = 0.0L;
        for (int j = 0; j < 2 * B; ++j) s += ctab[(size_t)a * 2 * B + j] * rad[(size_t)j * K + k];
        Kl[(size_t)a * K + k] = s / (2.0L * B);
      }
  }
}

// Q_lm P_lm(x) for l = m..B-1 (fixed m >= 0): the recurrence of Section 4,
// (l + 1 - m) P_{l+1,m} = (2l + 1) x P_lm - (l + m) P_{l-1,m}, seeded by
// P_mm = (-1)^m (2m-1)!! (1 - x^2)^{m/2}, then scaled by
// Q_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
static void legendre_normalised(int B, int m, long double x, long double *out) {
  const long double s = sqrtl(fmaxl(0.0L, 1.0L - x * x));
  long double pmm = 1.0L;
  for (int i = 1; i <= m; ++i) pmm *= -(2.0L * i - 1.0L) * s;
  long double pm1 = 0.0L, p0 = pmm;
  for (int l = m; l < B; ++l) {
    const long double Q = sqrtl((2.0L * l + 1.0L) / (4.0L * kPi) * expl(lgammal(l - m + 1.0L) - lgammal(l + m + 1.0L)));
    out[l - m] = Q * p0;
    const long double p1 = ((2.0L * l + 1.0L) * x * p0 - (l + m) * pm1) / (l + 1.0L - m);
    pm1 = p0;
    p0 = p1;
  }
}

void build_polar_table(int B, std::vector<long double> &out, std::vector<int64_t> &off) {
  off.assign(B + 1, 0);
  for (int m = 0; m < B; ++m) off[m + 1] = off[m] + (int64_t)B * (B - m);
  out.assign(off[B], 0.0L);
  std::vector<long double> leg((size_t)2 * B * B);
  std::vector<long double> ctab((size_t)2 * B * B), stab((size_t)2 * B * B);  // cos, sin(k1 w_j)
  for (int k1 = 0; k1 < B; ++k1)
    for (int j = 0; j < 2 * B; ++j) {
      ctab[(size_t)k1 * 2 * B + j] = cosl(k1 * node(B, j));
      stab[(size_t)k1 * 2 * B + j] = sinl(k1 * node(B, j));
    }
  for (int m = 0; m < B; ++m) {
    const int K = B - m;
    for (int j = 0; j < 2 * B; ++j) legendre_normalised(B, m, cosl(node(B, j)), leg.data() + (size_t)j * K);
    long double *Km = out.data() + off[m];
    for (int k1 = 0; k1 < B; ++k1)
      for (int c = 0; c < K; ++c) {
        const long double *tr = ((m & 1) ? stab.data() : ctab.data()) + (size_t)k1 * 2 * B;
        long double s = 0.0L;
        for (int j = 0; j < 2 * B; ++j) s += tr[j] * leg[(size_t)j * K + c];
        Km[(size_t)k1 * K + c] = s / (2.0L * B);
      }
  }
}

// Deconvolution with the Gaussian window of Def. 2.5 (Lemma 2.6):
// dc_j[kappa] = (2 pi lambda)^{-1/2} / phi_kappa, phi_kappa = exp(-2 lambda (pi kappa / N_j)^2),
// for kappa in I_{n_j}.  The product over the three dimensions is the net
// factor between eta_k and the coefficients transformed by the FFT once the
// constants (2 pi)^d, (sigma n)^{-d} and the window's (sigma n / 2 pi)^d
// normalisation are collected (Section 2).
void build_deconv(const Plan &p, std::vector<long double> &out) {
  out.clear();
  const long double lam = p.lambda;
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < p.n[j]; ++i) {
      const long double kap = i - p.n[j] / 2;
      const long double x = kPi * kap / p.N[j];
      out.push_back(expl(2.0L * lam * x * x) / sqrtl(2.0L * kPi * lam));
    }
}

void build_twiddles(int L, int sign, std::vector<long double> &re, std::vector<long double> &im) {
  re.resize(L);
  im.resize(L);
  for (int t = 0; t < L; ++t) {
    const long double a = 2.0L * kPi * t / L;
    re[t] = cosl(a);
    im[t] = sign * sinl(a);
  }
}

}  // namespace sgl
