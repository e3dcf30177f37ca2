"""Pins of the direct oracle (exact NDSGLFT, Def. 1.3) against facts that do
not come from the oracle itself: closed forms of low-order basis functions,
orthonormality (Thm. 1.2) under an exact product quadrature, scipy's special
functions, symmetry invariants and the adjoint identity."""
import math

import numpy as np
import pytest
from scipy import special as sp

import oracle
from oracle import stepwise as sw
from tests import workloads as wl

PI34 = math.pi ** -0.75


def _pts(M, seed):
    return wl.gaussian_points(M, seed)


def test_closed_forms_low_order():
    """H_100, H_200, H_210, H_21+-1 written out from Def. 1.1 by hand."""
    pts = _pts(25, 1)
    for x, y, z in pts:
        r2 = x * x + y * y + z * z
        h = oracle.basis(2, [x, y, z])
        want = {
            (1, 0, 0): PI34,
            (2, 0, 0): PI34 * math.sqrt(2.0 / 3.0) * (1.5 - r2),
            (2, 1, -1): PI34 * (x - 1j * y),
            (2, 1, 0): math.sqrt(2.0) * PI34 * z,
            (2, 1, 1): -PI34 * (x + 1j * y),
        }
        for (n, l, m), v in want.items():
            assert abs(h[sw.mu_of(n, l, m)] - v) < 1e-14


def test_bandwidth_one_is_constant():
    pts = _pts(50, 2)
    fh = np.array([0.7 - 0.3j])
    f = oracle.direct_forward(1, pts, fh)
    assert np.allclose(f, fh[0] * PI34, rtol=0, atol=1e-15)


def _gram(B, long_double=False):
    """Gram matrix of the H_mu under Gauss-Laguerre(alpha=1/2, B) in s = r^2,
    Gauss-Legendre(B) in cos(theta) and the trapezoid rule (2B-1) in phi.
    Exact for bandwidth B (Thm. 1.2 then says it is the identity)."""
    s, ws = sp.roots_genlaguerre(B, 0.5)
    xg, wg = np.polynomial.legendre.leggauss(B)
    P = 2 * B - 1
    nc = wl.num_coeffs(B)
    G = np.zeros((nc, nc), dtype=np.complex128)
    for sk, wk in zip(s, ws):
        r = math.sqrt(sk)
        for xj, wj in zip(xg, wg):
            st = math.sqrt(max(0.0, 1 - xj * xj))
            for p in range(P):
                ph = 2 * math.pi * p / P
                pt = [r * st * math.cos(ph), r * st * math.sin(ph), r * xj]
                h = oracle.basis(B, pt, long_double=long_double)
                G += (wk / 2) * wj * (2 * math.pi / P) * np.outer(h, h.conj())
    return G


@pytest.mark.parametrize("B", [2, 4])
def test_orthonormal_under_exact_quadrature(B):
    G = _gram(B)
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


def test_matches_scipy_special_functions():
    """Same basis built from scipy's eval_genlaguerre and sph_harm_y."""
    B = 7
    pts = _pts(40, 3)
    ref = sw.sgl_basis(B, pts)
    for i, p in enumerate(pts):
        h = oracle.basis(B, p)
        assert np.abs(h - ref[i]).max() < 1e-12 * max(1.0, np.abs(ref[i]).max())


def test_parity_and_z_rotation():
    """H(-x) = (-1)^l H(x);  H(R_z(a) x) = e^{i m a} H(x)."""
    B = 9
    ns, ls, ms = sw.coeff_table(B)
    a = 0.731
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    for p in _pts(10, 4):
        h = oracle.basis(B, p)
        assert np.abs(oracle.basis(B, -p) - (-1.0) ** ls * h).max() < 1e-12
        assert np.abs(oracle.basis(B, Rz @ p) - np.exp(1j * ms * a) * h).max() < 1e-12


def test_adjoint_identity():
    B = 10
    pts = _pts(300, 5)
    fh = wl.coefficients(B, 6)
    y = wl.samples(300, 7)
    f = oracle.direct_forward(B, pts, fh)
    g = oracle.direct_adjoint(B, pts, y)
    lhs = np.vdot(y, f)  # <Lambda fhat, y>
    rhs = np.vdot(g, fh)  # <fhat, Lambda^H y>
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_forward_is_sum_over_basis():
    """Forward == explicit matrix Lambda (scipy basis) times fhat."""
    B = 6
    pts = _pts(60, 8)
    fh = wl.coefficients(B, 9)
    Lam = sw.sgl_basis(B, pts)
    assert np.abs(oracle.direct_forward(B, pts, fh) - Lam @ fh).max() < 1e-12
    y = wl.samples(60, 10)
    assert np.abs(oracle.direct_adjoint(B, pts, y) - Lam.conj().T @ y).max() < 1e-12


def test_long_double_agrees_with_double():
    """The paper ran its recurrences in 80-bit long double; at B=24 and r up to
    ~4 both precisions agree to ~1e-13 relative."""
    B = 24
    pts = _pts(400, 11)
    fh = wl.coefficients(B, 12)
    f64 = oracle.direct_forward(B, pts, fh)
    f80 = oracle.direct_forward(B, pts, fh, long_double=True)
    assert np.linalg.norm(f64 - f80) / np.linalg.norm(f80) < 1e-13


def test_thread_count_invariance():
    B = 8
    pts = _pts(500, 13)
    fh = wl.coefficients(B, 14)
    a = oracle.direct_forward(B, pts, fh, nthreads=1)
    b = oracle.direct_forward(B, pts, fh, nthreads=4)
    assert np.array_equal(a, b)
