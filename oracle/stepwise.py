"""ORACLE -- test infrastructure only (see ``oracle/__init__.py``).

The fast SGL Fourier transform for scattered data (NFSGLFT) and its adjoint,
taken step by step in the paper's order and notation, in plain numpy/scipy at
float64, with every matrix of the factorization built explicitly:

  Lambda = N (1 (x) Z_B^T)(1 (x) X_B^T)(1 (x) (+)_m W_m D C~)(1 (x) (+)_m L~_m^T)
             U_B^T (1 (x) A_B D C~)((+)_l R~_l) S_B^T                (Thm. 6.2)

and the adjoint as the reversed product of conjugate transposes (Cor. 6.3).
The final factor N is either the exact NDFT (Def. 2.4) or the Gaussian NFFT of
Section 2 (Def. 2.5, Lemma 2.6, window truncation eq. (2.x) "nfft_psi").

Special functions come from scipy (generalised Laguerre polynomials, Gamma,
spherical harmonics), i.e. an implementation independent of the C oracle.
Meant for small bandwidths (B <= 16) and modest numbers of points.

Readings where the paper is ambiguous (each listed in the design doc):
  * mu -> (n,l,m): the closed form of eq. (1.1) is evaluated in float64 and
    then corrected by exact integer arithmetic (it lands exactly on block
    boundaries, where floor() can go either way).
  * V_B uses (2j+1)pi/(4B), the polar nodes of the derivation.
  * Z_B pads m = 1-B..B-1 into kappa_2 in I_{4B} (or I_{2B} for the reduced
    grid of Remark 8.1).
  * Window taps: for each dimension the integers l with u - q < l <= u + q
    (u = N t / 2 pi), i.e. exactly 2q taps; the closed box of the definition
    differs only when u - q is an integer, and the truncation-error term in
    the proof of Thm. 2.7 already counts those boundary taps as dropped.
"""
import math

import numpy as np
from scipy import special as sp

# ----------------------------------------------------------------------------
# Index linearisation (Section 1)
# ----------------------------------------------------------------------------


def num_coeffs(B):
    return B * (B + 1) * (2 * B + 1) // 6


def mu_of(n, l, m):
    """mu = n(n-1)(2n-1)/6 + l(l+1) + m  (Section 1)."""
    return n * (n - 1) * (2 * n - 1) // 6 + l * (l + 1) + m


def nlm_of(mu):
    """Inverse map of eq. (1.1): closed form for n, then exact integer fix-up."""
    if mu == 0:
        return 1, 0, 0
    n = int(math.floor(math.cosh(math.acosh(36.0 * math.sqrt(3.0) * mu) / 3.0) / math.sqrt(3.0) + 0.5))
    # exact correction: n is the largest integer with n(n-1)(2n-1)/6 <= mu
    while n * (n - 1) * (2 * n - 1) // 6 > mu:
        n -= 1
    while (n + 1) * n * (2 * n + 1) // 6 <= mu:
        n += 1
    rem = mu - n * (n - 1) * (2 * n - 1) // 6
    l = math.isqrt(rem)
    m = rem - l * (l + 1)
    return n, l, m


def coeff_table(B):
    """Arrays n, l, m indexed by mu."""
    t = np.array([nlm_of(mu) for mu in range(num_coeffs(B))], dtype=np.int64)
    return t[:, 0], t[:, 1], t[:, 2]


# ----------------------------------------------------------------------------
# Special functions (Def. 1.1, Section 4)
# ----------------------------------------------------------------------------


def N_nl(n, l):
    """N_nl = sqrt(2 (n-l-1)! / Gamma(n+1/2))."""
    return math.sqrt(2.0) * math.exp(0.5 * (sp.gammaln(n - l) - sp.gammaln(n + 0.5)))


def radial(n, l, r):
    """N_nl R_nl(r) = N_nl L_{n-l-1}^{(l+1/2)}(r^2) r^l."""
    r = np.asarray(r, dtype=np.float64)
    return N_nl(n, l) * sp.eval_genlaguerre(n - l - 1, l + 0.5, r * r) * r ** l


def Q_P(l, m, ct_theta):
    """Q_lm P_lm(cos theta), i.e. Y_lm(theta, 0); P_lm with the (-1)^m factor."""
    th = np.arccos(np.clip(ct_theta, -1.0, 1.0))
    return np.real(sp.sph_harm_y(l, m, th, 0.0))


def Q_lm(l, m):
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.exp(sp.gammaln(l - m + 1) - sp.gammaln(l + m + 1)))


def sgl_basis(B, points):
    """Lambda itself (Def. 1.3), M x Nc, for small cases."""
    r, th, ph = spherical(points)
    ns, ls, ms = coeff_table(B)
    out = np.empty((len(r), len(ns)), dtype=np.complex128)
    for mu, (n, l, m) in enumerate(zip(ns, ls, ms)):
        out[:, mu] = radial(n, l, r) * sp.sph_harm_y(l, m, th, ph)
    return out


def sgl_basis_grad(B, points):
    """d H_nlm(x) / d x_c for c = 0, 1, 2: array (3, M, Nc).

    Chain rule through (r, theta, phi): the radial factor N_nl L_k^(a)(r^2) r^l
    (k = n-l-1, a = l+1/2) differentiates with d/dt L_k^(a)(t) = -L_{k-1}^(a+1)(t);
    the angular factor Y_lm with scipy's derivatives in theta and phi.
    Undefined on the z axis and at the origin, where phi or theta is.
    """
    p = np.asarray(points, dtype=np.float64)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    r, th, ph = spherical(p)
    rxy = np.hypot(x, y)
    dr = np.stack([x / r, y / r, z / r])
    dth = np.stack([x * z / (r * r * rxy), y * z / (r * r * rxy), -rxy / (r * r)])
    dph = np.stack([-y / (rxy * rxy), x / (rxy * rxy), np.zeros_like(x)])
    ns, ls, ms = coeff_table(B)
    out = np.empty((3, len(r), len(ns)), dtype=np.complex128)
    for mu, (n, l, m) in enumerate(zip(ns, ls, ms)):
        k, a = n - l - 1, l + 0.5
        t = r * r
        L = sp.eval_genlaguerre(k, a, t)
        dL = -sp.eval_genlaguerre(k - 1, a + 1, t) if k >= 1 else np.zeros_like(t)
        c = N_nl(n, l)
        R = c * L * r ** l
        dR = c * (2 * r * dL * r ** l + (l * L * r ** (l - 1) if l > 0 else 0.0))
        Y, dY = sp.sph_harm_y(l, m, th, ph, diff_n=1)  # dY: (M, 2) = d/dtheta, d/dphi
        dYth, dYph = dY[..., 0], dY[..., 1]
        out[:, :, mu] = dR * Y * dr + R * dYth * dth + R * dYph * dph
    return out


def forward_grad(B, points, fhat):
    """d f(x_i) / d x_ic of f = Lambda fhat (Def. 1.3), shape (M, 3), complex."""
    G = sgl_basis_grad(B, points)
    return np.einsum("cmn,n->mc", G, np.asarray(fhat, dtype=np.complex128))


# ----------------------------------------------------------------------------
# DCT (Def. 3.1)
# ----------------------------------------------------------------------------


def omega(n):
    """omega_j = (2j+1) pi / (2n), j < n."""
    return (2 * np.arange(n) + 1) * np.pi / (2 * n)


def D_mat(n):
    d = np.full(n, math.sqrt(2.0 / n))
    d[0] = 1.0 / math.sqrt(n)
    return np.diag(d)


def C_mat(n):
    w = omega(n)
    return np.cos(np.outer(np.arange(n), w))


def Ctilde(n):
    """The DCT C~_n = D_n C_n."""
    return D_mat(n) @ C_mat(n)


# ----------------------------------------------------------------------------
# Matrices of Theorem 6.2
# ----------------------------------------------------------------------------


def R_l(l, B, rho):
    """R_l in R^{2B x (B-l)}: N_nl R_nl(rho (1 + cos omega_j) / 2)."""
    w = omega(2 * B)
    rj = rho * (1 + np.cos(w)) / 2
    return np.stack([radial(n, l, rj) for n in range(l + 1, B + 1)], axis=1)


def Ltilde_T(m, B):
    """L~_m^T = {1 or V_B} L_m^T diag(Q_lm), in R^{2B x (B-|m|)}."""
    w = omega(2 * B)  # = (2j+1) pi / (4B)
    cols = [Q_P(l, m, np.cos(w)) for l in range(abs(m), B)]
    M = np.stack(cols, axis=1)
    if m % 2:
        M = M / np.sin(w)[:, None]  # V_B
    return M


def A_B(B):
    """A_B in R^{4B x 2B}; rows kappa = -2B..2B-1, columns kappa' = 0..2B-1."""
    A = np.zeros((4 * B, 2 * B))
    for kap in range(-2 * B, 2 * B):
        row = kap + 2 * B
        if kap == 0:
            A[row, 0] = 1.0
        elif abs(kap) < 2 * B:
            A[row, abs(kap)] = 0.5
    return A


def W_m(m, B):
    """W_m: A_B for even m; for odd m the matrix of eq. nfsglft_a_zeta_odd."""
    if m % 2 == 0:
        return A_B(B).astype(np.complex128)
    W = np.zeros((4 * B, 2 * B), dtype=np.complex128)
    for kap in range(-2 * B, 2 * B):
        row = kap + 2 * B
        a = abs(kap)
        if kap == 0 or kap == -2 * B:
            continue
        s = np.sign(kap) / 4j
        if a == 1:
            W[row, 0] += 2 * s
            W[row, 2] -= s
        elif a < 2 * B - 2:
            W[row, a - 1] += s
            W[row, a + 1] -= s
        else:  # 2B-2 <= |kappa| < 2B
            W[row, a - 1] += s
    return W


# ----------------------------------------------------------------------------
# Points (Section 6, eq. x_tilde)
# ----------------------------------------------------------------------------


def spherical(points):
    p = np.asarray(points, dtype=np.float64)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    rxy = np.hypot(x, y)
    r = np.hypot(rxy, z)
    th = np.arctan2(rxy, z)
    ph = np.mod(np.arctan2(y, x), 2 * np.pi)
    return r, th, ph


def rho_of(points):
    """rho = max_i r_i (eq. nfsglft_rho); 1 if every point is the origin."""
    r = spherical(points)[0]
    m = float(r.max()) if len(r) else 0.0
    return m if m > 0 else 1.0


def x_tilde(points, rho):
    """[arccos gamma(r), theta, phi] in T^3 with gamma(r) = (2r - rho)/rho."""
    r, th, ph = spherical(points)
    g = np.clip((2 * r - rho) / rho, -1.0, 1.0)
    return np.stack([np.arccos(g), th, ph], axis=1)


# ----------------------------------------------------------------------------
# Conversion: fhat -> eta (all factors of Thm. 6.2 right of N)
# ----------------------------------------------------------------------------


def conversion(B, fhat, rho, reduced=True):
    """Trigonometric coefficients eta_k of eq. nfsglft_nfft.

    Returns a dense array eta[k0 + 2B, k1 + n1/2, k2 + n2/2] on the grid
    I_{4B} x I_{4B} x I_{4B}, or the reduced 4B x 2B x 2B grid (Remark 8.1).
    """
    fhat = np.asarray(fhat, dtype=np.complex128)
    ns, ls, ms = coeff_table(B)
    CT = Ctilde(2 * B)
    D = D_mat(2 * B)
    AB = A_B(B)
    # beta[kappa0, l, m] via (1 (x) A_B D C~)(+) R~_l S_B^T
    beta = np.zeros((4 * B, B, 2 * B - 1), dtype=np.complex128)  # m index m+B-1
    for l in range(B):
        R = R_l(l, B, rho)
        K = AB @ D @ CT @ R  # 4B x (B-l)
        for m in range(-l, l + 1):
            F = np.array([fhat[mu_of(n, l, m)] for n in range(l + 1, B + 1)])
            beta[:, l, m + B - 1] = K @ F
    # U_B^T reorders to (kappa0, m, l); then per (kappa0, m) the spherical part
    zeta = np.zeros((4 * B, 4 * B, 2 * B - 1), dtype=np.complex128)  # [k0, k1, m]
    for m in range(1 - B, B):
        LT = Ltilde_T(m, B)  # 2B x (B-|m|)
        P = W_m(m, B) @ D @ CT @ LT  # 4B x (B-|m|)
        bm = beta[:, abs(m):, m + B - 1]  # 4B(k0) x (B-|m|)
        zeta[:, :, m + B - 1] = bm @ P.T
    # X_B^T, Z_B^T: place m into kappa_2
    n12 = 2 * B if reduced else 4 * B
    eta = np.zeros((4 * B, n12, n12), dtype=np.complex128)
    k1lo = 2 * B - n12 // 2  # rows of zeta kept
    eta[:, :, n12 // 2 - (B - 1): n12 // 2 + B] = zeta[:, k1lo: k1lo + n12, :]
    return eta


def conversion_adjoint(B, eta, rho):
    """Adjoint of ``conversion`` (Cor. 6.3), from eta on either grid."""
    eta = np.asarray(eta, dtype=np.complex128)
    n12 = eta.shape[1]
    ns, ls, ms = coeff_table(B)
    CT = Ctilde(2 * B)
    D = D_mat(2 * B)
    AB = A_B(B)
    zeta = np.zeros((4 * B, 4 * B, 2 * B - 1), dtype=np.complex128)
    k1lo = 2 * B - n12 // 2
    zeta[:, k1lo: k1lo + n12, :] = eta[:, :, n12 // 2 - (B - 1): n12 // 2 + B]
    beta = np.zeros((4 * B, B, 2 * B - 1), dtype=np.complex128)
    for m in range(1 - B, B):
        LT = Ltilde_T(m, B)
        # (W_m D C~ L~_m^T)^H = L~_m C~^T D^T W_m^H  (C~^{-1} = C~^T, Lemma 3.3)
        P = W_m(m, B) @ D @ CT @ LT
        beta[:, abs(m):, m + B - 1] = zeta[:, :, m + B - 1] @ P.conj()
    fh = np.zeros(num_coeffs(B), dtype=np.complex128)
    for l in range(B):
        R = R_l(l, B, rho)
        K = AB @ D @ CT @ R
        for m in range(-l, l + 1):
            v = K.T @ beta[:, l, m + B - 1]
            for n in range(l + 1, B + 1):
                fh[mu_of(n, l, m)] = v[n - l - 1]
    return fh


# ----------------------------------------------------------------------------
# NDFT (Def. 2.4) and Gaussian NFFT (Section 2)
# ----------------------------------------------------------------------------


def _kvec(n):
    return np.arange(-n // 2, n // 2)


def ndft(eta, t):
    """p(t_i) = sum_{k in I_n} eta_k e^{i <k, t_i>} (exact)."""
    n0, n1, n2 = eta.shape
    e0 = np.exp(1j * np.outer(t[:, 0], _kvec(n0)))
    e1 = np.exp(1j * np.outer(t[:, 1], _kvec(n1)))
    e2 = np.exp(1j * np.outer(t[:, 2], _kvec(n2)))
    return np.einsum("pa,pb,pc,abc->p", e0, e1, e2, eta, optimize=True)


def ndft_adjoint(y, t, shape):
    n0, n1, n2 = shape
    e0 = np.exp(-1j * np.outer(t[:, 0], _kvec(n0)))
    e1 = np.exp(-1j * np.outer(t[:, 1], _kvec(n1)))
    e2 = np.exp(-1j * np.outer(t[:, 2], _kvec(n2)))
    return np.einsum("p,pa,pb,pc->abc", np.asarray(y, dtype=np.complex128), e0, e1, e2, optimize=True)


def nfft_lambda(sigma, q):
    """lambda = sigma q / ((2 sigma - 1) pi)  (Thm. 2.7)."""
    return sigma * q / ((2 * sigma - 1) * np.pi)


def _phi_hat(kappa, Nj, lam):
    """phi_kappa = exp(-2 lambda (pi kappa / sigma n)^2)  (Lemma 2.6)."""
    return np.exp(-2.0 * lam * (np.pi * kappa / Nj) ** 2)


def _window_taps(tj, Nj, q, lam):
    """Taps and values of the 1D factor of psi~ at t - 2 pi l / N (Def. 2.5)."""
    u = Nj * tj / (2 * np.pi)
    first = np.floor(u - q).astype(np.int64) + 1  # u - q < l <= u + q
    ls = first[:, None] + np.arange(2 * q)[None, :]
    xi = tj[:, None] - 2 * np.pi * ls / Nj
    phi = (1.0 / np.sqrt(2 * np.pi * lam)) * (Nj / (2 * np.pi)) * np.exp(
        -((Nj / (2 * np.pi)) ** 2) * xi ** 2 / (2 * lam))
    return np.mod(ls, Nj), phi


def nfft(eta, t, sigma, q, chunk=512):
    """Gaussian NFFT of Section 2 on the (possibly anisotropic) grid eta.shape."""
    n = eta.shape
    N = tuple(sigma * nj for nj in n)
    lam = nfft_lambda(sigma, q)
    # beta_k = omega_k / phi~_k on I_n, zero elsewhere in I_{sigma n}
    ks = [_kvec(nj) for nj in n]
    phit = (2 * np.pi) ** -3 * (_phi_hat(ks[0], N[0], lam)[:, None, None] *
                                _phi_hat(ks[1], N[1], lam)[None, :, None] *
                                _phi_hat(ks[2], N[2], lam)[None, None, :])
    beta = np.zeros(N, dtype=np.complex128)
    idx = np.ix_(np.mod(ks[0], N[0]), np.mod(ks[1], N[1]), np.mod(ks[2], N[2]))
    beta[idx] = eta / phit
    # alpha_l = (sigma n)^{-d} sum_k beta_k e^{+2 pi i <k,l>/sigma n}  (inverse of F)
    alpha = np.fft.ifftn(beta)
    out = np.empty(t.shape[0], dtype=np.complex128)
    for s in range(0, t.shape[0], chunk):
        tt = t[s:s + chunk]
        i0, w0 = _window_taps(tt[:, 0], N[0], q, lam)
        i1, w1 = _window_taps(tt[:, 1], N[1], q, lam)
        i2, w2 = _window_taps(tt[:, 2], N[2], q, lam)
        g = alpha[i0[:, :, None, None], i1[:, None, :, None], i2[:, None, None, :]]
        out[s:s + chunk] = np.einsum("pa,pb,pc,pabc->p", w0, w1, w2, g, optimize=True)
    return out


def nfft_adjoint(y, t, shape, sigma, q, chunk=512):
    """Adjoint Gaussian NFFT: transposes of the factors of ``nfft`` in reverse."""
    n = shape
    N = tuple(sigma * nj for nj in n)
    lam = nfft_lambda(sigma, q)
    y = np.asarray(y, dtype=np.complex128)
    grid = np.zeros(N, dtype=np.complex128)
    for s in range(0, t.shape[0], chunk):
        tt = t[s:s + chunk]
        i0, w0 = _window_taps(tt[:, 0], N[0], q, lam)
        i1, w1 = _window_taps(tt[:, 1], N[1], q, lam)
        i2, w2 = _window_taps(tt[:, 2], N[2], q, lam)
        v = (y[s:s + chunk, None, None, None] * w0[:, :, None, None] * w1[:, None, :, None] *
             w2[:, None, None, :])
        np.add.at(grid, (np.broadcast_to(i0[:, :, None, None], v.shape),
                         np.broadcast_to(i1[:, None, :, None], v.shape),
                         np.broadcast_to(i2[:, None, None, :], v.shape)), v)
    # adjoint of ifftn: (sigma n)^{-d} F, F with e^{-2 pi i <k,l>/sigma n}
    bh = np.fft.fftn(grid) / np.prod(N)
    ks = [_kvec(nj) for nj in n]
    phit = (2 * np.pi) ** -3 * (_phi_hat(ks[0], N[0], lam)[:, None, None] *
                                _phi_hat(ks[1], N[1], lam)[None, :, None] *
                                _phi_hat(ks[2], N[2], lam)[None, None, :])
    idx = np.ix_(np.mod(ks[0], N[0]), np.mod(ks[1], N[1]), np.mod(ks[2], N[2]))
    return bh[idx] / phit


def nfft_error_bound(sigma, q, d=3):
    """The factor multiplying ||w||_1 in Thm. 2.7 (requires sigma >= (sqrt d + 1)/2)."""
    e = np.exp(-q * np.pi * (1 - (1 + d / (2 * sigma - 1)) / (2 * sigma)))
    c = ((2 ** d - 1) * (2 + 1 / (np.pi * q)) ** d +
         (3 ** d - 1) / q ** (d / 2) *
         (np.sqrt((2 * sigma - 1) / (2 * sigma)) + np.sqrt(2 * sigma / (2 * sigma - 1)) / (2 * np.pi)) ** d)
    return c * e


# ----------------------------------------------------------------------------
# Full transforms
# ----------------------------------------------------------------------------


def forward(B, fhat, points, rho=None, sigma=2, q=None, exact=False, reduced=True):
    """NFSGLFT: conversion to eta, then the NDFT (exact=True) or the NFFT."""
    rho = rho_of(points) if rho is None else rho
    eta = conversion(B, fhat, rho, reduced=reduced)
    t = x_tilde(points, rho)
    if exact:
        return ndft(eta, t)
    return nfft(eta, t, sigma, q)


def adjoint(B, y, points, rho=None, sigma=2, q=None, exact=False, reduced=True):
    rho = rho_of(points) if rho is None else rho
    t = x_tilde(points, rho)
    shape = (4 * B, 2 * B, 2 * B) if reduced else (4 * B, 4 * B, 4 * B)
    eta = ndft_adjoint(y, t, shape) if exact else nfft_adjoint(y, t, shape, sigma, q)
    return conversion_adjoint(B, eta, rho)
