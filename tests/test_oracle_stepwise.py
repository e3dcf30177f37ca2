"""Pins of the stepwise oracle (the paper's fast algorithm in its own order):
the DCT lemmas of Section 3, the Chebyshev-to-exponential matrices A_B and W_m,
exactness of the factorization (Thm. 6.2 with the exact NDFT equals the direct
sum), the adjoint factorization (Cor. 6.3), and the NFFT error theory of
Thm. 2.7."""
import math

import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import stepwise as sw
from tests import workloads as wl


# ---------------------------------------------------------------- index map


def test_mu_roundtrip_and_order():
    B = 40
    mu = 0
    for n in range(1, B + 1):
        for l in range(n):
            for m in range(-l, l + 1):
                assert sw.mu_of(n, l, m) == mu
                assert sw.nlm_of(mu) == (n, l, m)
                mu += 1
    assert mu == sw.num_coeffs(B)


def test_mu_closed_form_needs_integer_fixup():
    """eq. (1.1) evaluated in float64 lands exactly on the block boundaries
    mu = n(n-1)(2n-1)/6, where floor() can return n-1 (reading G2)."""
    bad = 0
    for n in range(2, 200):
        mu = n * (n - 1) * (2 * n - 1) // 6
        naive = math.floor(math.cosh(math.acosh(36 * math.sqrt(3) * mu) / 3) / math.sqrt(3) + 0.5)
        bad += naive != n
        assert sw.nlm_of(mu) == (n, 0, 0)
    assert bad > 0


# ---------------------------------------------------------------- DCT (Section 3)


@pytest.mark.parametrize("n", [4, 7, 16])
def test_dct_orthogonal_and_matches_dct2(n):
    C = sw.Ctilde(n)
    assert np.abs(C.T @ C - np.eye(n)).max() < 1e-14  # Lemma 3.3
    x = np.random.default_rng(n).standard_normal(n)
    assert np.abs(C @ x - scipy.fft.dct(x, type=2, norm="ortho")).max() < 1e-14


def test_dct_yields_chebyshev_coefficients():
    """Lemma 3.5: D_n C~_n [p(cos w_j)] are the Chebyshev coefficients of p."""
    n = 12
    a = np.random.default_rng(1).standard_normal(n)
    w = sw.omega(n)
    p = np.polynomial.chebyshev.chebval(np.cos(w), a)
    assert np.abs(sw.D_mat(n) @ sw.Ctilde(n) @ p - a).max() < 1e-13


def test_A_B_is_cosine_to_exponential():
    B = 6
    alpha = np.random.default_rng(2).standard_normal(2 * B)
    alpha[-1] = 0.0
    beta = sw.A_B(B) @ alpha
    k = np.arange(-2 * B, 2 * B)
    for om in np.linspace(0, math.pi, 9):
        lhs = np.sum(beta * np.exp(1j * k * om))
        rhs = np.sum(alpha * np.cos(np.arange(2 * B) * om))
        assert abs(lhs - rhs) < 1e-13


def test_W_odd_is_sine_cosine_to_exponential():
    """eq. nfsglft_a_zeta_odd: sum_k zeta_k e^{ik w} = sum_k eps_k sin(w) cos(k w)."""
    B = 6
    eps = np.random.default_rng(3).standard_normal(2 * B)
    eps[2 * B - 1] = 0.0  # the expansion runs to 2B-2
    zeta = sw.W_m(1, B) @ eps
    k = np.arange(-2 * B, 2 * B)
    for om in np.linspace(0.1, 3.0, 7):
        lhs = np.sum(zeta * np.exp(1j * k * om))
        rhs = np.sum(eps * math.sin(om) * np.cos(np.arange(2 * B) * om))
        assert abs(lhs - rhs) < 1e-13


# ---------------------------------------------------------------- factorization


@pytest.mark.parametrize("B", [2, 3, 5, 8])
@pytest.mark.parametrize("reduced", [True, False])
def test_factorization_with_ndft_is_exact(B, reduced):
    """Thm. 6.2 with the exact NDFT reproduces the direct sum to roundoff."""
    pts = wl.gaussian_points(150, 20 + B)
    fh = wl.coefficients(B, 21 + B)
    f0 = oracle.direct_forward(B, pts, fh)
    f1 = sw.forward(B, fh, pts, exact=True, reduced=reduced)
    assert np.linalg.norm(f1 - f0) / np.linalg.norm(f0) < 1e-13
    y = wl.samples(150, 22 + B)
    g0 = oracle.direct_adjoint(B, pts, y)
    g1 = sw.adjoint(B, y, pts, exact=True, reduced=reduced)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 1e-13


def test_reduced_grid_drops_only_zeros():
    """Remark 8.1: eta vanishes outside 4B x 2B x 2B (up to roundoff)."""
    B = 7
    fh = wl.coefficients(B, 30)
    full = sw.conversion(B, fh, 3.5, reduced=False)
    red = sw.conversion(B, fh, 3.5, reduced=True)
    inner = full[:, B:3 * B, B:3 * B]
    assert np.array_equal(inner, red)
    outer = np.abs(full).sum() - np.abs(inner).sum()
    assert outer < 1e-13 * np.abs(full).sum()
    # kappa0 = +-(2B-1) and kappa1 = -B rows are zero too (degree argument)
    assert np.abs(red[[1, 4 * B - 1]]).max() < 1e-13 * np.abs(red).max()
    assert np.abs(red[:, 0]).max() < 1e-13 * np.abs(red).max()


def test_conversion_adjoint_identity():
    B = 6
    rho = 3.1
    fh = wl.coefficients(B, 31)
    eta = np.random.default_rng(32).standard_normal((4 * B, 2 * B, 2 * B)) * (1 + 1j)
    lhs = np.vdot(eta, sw.conversion(B, fh, rho))
    rhs = np.vdot(sw.conversion_adjoint(B, eta, rho), fh)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# ---------------------------------------------------------------- NFFT (Section 2)


def _random_trig(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_nfft_delta_is_one():
    """omega = delta_0 gives p == 1; the NFFT reproduces it within the bound."""
    shape = (8, 4, 4)
    eta = np.zeros(shape, dtype=np.complex128)
    eta[4, 2, 2] = 1.0
    t = np.random.default_rng(40).uniform(0, 2 * np.pi, (100, 3))
    for q in (4, 8):
        s = sw.nfft(eta, t, 2, q)
        assert np.abs(s - 1).max() < sw.nfft_error_bound(2, q)


def test_nfft_within_theorem_bound_and_decays():
    """Thm. 2.7: |p - s| <= ||w||_1 * bound(sigma, q); observation O1."""
    shape = (16, 8, 8)
    eta = _random_trig(shape, 41)
    t = np.random.default_rng(42).uniform(0, 2 * np.pi, (300, 3))
    p = sw.ndft(eta, t)
    w1 = np.abs(eta).sum()
    errs = []
    for q in range(2, 11):
        e = np.abs(sw.nfft(eta, t, 2, q) - p).max()
        assert e <= w1 * sw.nfft_error_bound(2, q)
        errs.append(e)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    assert errs[-1] < 1e-8 * np.abs(p).max()


def test_nfft_adjoint_identity():
    shape = (16, 8, 8)
    eta = _random_trig(shape, 43)
    t = np.random.default_rng(44).uniform(0, 2 * np.pi, (200, 3))
    y = wl.samples(200, 45)
    lhs = np.vdot(y, sw.nfft(eta, t, 2, 5))
    rhs = np.vdot(sw.nfft_adjoint(y, t, shape, 2, 5), eta)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_nfsglft_error_small_at_q12():
    """Fast forward and adjoint against the direct sum at B=8, q=12."""
    B = 8
    pts = wl.gaussian_points(400, 50)
    fh = wl.coefficients(B, 51, 2.0)
    f0 = oracle.direct_forward(B, pts, fh)
    f1 = sw.forward(B, fh, pts, q=12)
    assert np.linalg.norm(f1 - f0) / np.linalg.norm(f0) < 1e-8
    y = wl.samples(400, 52)
    g0 = oracle.direct_adjoint(B, pts, y)
    g1 = sw.adjoint(B, y, pts, q=12)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 1e-8


def test_nfsglft_error_decays_in_q():
    """Observation O1 for the whole transform."""
    B = 6
    pts = wl.ball_points(200, 3.0, 53)
    fh = wl.coefficients_uniform(B, 54)
    f0 = oracle.direct_forward(B, pts, fh)
    errs = [np.abs(sw.forward(B, fh, pts, q=q) - f0).max() for q in (3, 5, 7, 9)]
    assert all(errs[i + 1] < 0.2 * errs[i] for i in range(len(errs) - 1))


# ------------------------------------------------------------ gradient in x


def test_basis_grad_matches_central_differences():
    """d H / d x against central differences of the basis itself (B = 4)."""
    B = 4
    pts = np.array([[0.3, -0.5, 0.7], [-1.1, 0.4, -0.2], [0.6, 0.9, 1.3]])
    G = sw.sgl_basis_grad(B, pts)
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (sw.sgl_basis(B, pts + e) - sw.sgl_basis(B, pts - e)) / (2 * h)
        assert np.abs(G[c] - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())


def test_basis_grad_closed_forms():
    """H_100 is constant; H_210 = N_21 sqrt(3/(4 pi)) z; H_211 = -N_21 sqrt(3/(8 pi)) (x + i y)
    (Condon-Shortley phase of P_lm in Rodrigues form)."""
    pts = np.array([[0.3, -0.5, 0.7], [-1.1, 0.4, -0.2]])
    G = sw.sgl_basis_grad(2, pts)
    n21 = math.sqrt(2.0 / math.gamma(2.5))
    mu100, mu210, mu211 = sw.mu_of(1, 0, 0), sw.mu_of(2, 1, 0), sw.mu_of(2, 1, 1)
    assert np.abs(G[:, :, mu100]).max() < 1e-14
    c = n21 * math.sqrt(3.0 / (4 * math.pi))
    assert np.allclose(G[:, :, mu210], np.array([[0, 0], [0, 0], [c, c]]), atol=1e-13)
    c1 = -n21 * math.sqrt(3.0 / (8 * math.pi))
    assert np.allclose(G[:, :, mu211], np.array([[c1, c1], [1j * c1, 1j * c1], [0, 0]]), atol=1e-13)


def test_forward_grad_matches_direct_sum_differences():
    """Gradient of f = Lambda fhat against central differences of the exact
    direct sum (B = 6, long double build of the oracle library)."""
    B = 6
    rng = np.random.default_rng(3)
    pts = rng.standard_normal((5, 3)) * 0.7
    fh = wl.coefficients(B, 4)
    g = sw.forward_grad(B, pts, fh)
    h = 1e-5
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (oracle.direct_forward(B, pts + e, fh, long_double=True)
              - oracle.direct_forward(B, pts - e, fh, long_double=True)) / (2 * h)
        assert np.abs(g[:, c] - fd).max() < 1e-8 * np.abs(fd).max()
