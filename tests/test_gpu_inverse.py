"""Inverse transform (weighted CGNR over the plan's forward and adjoint).

Data are exact samples of a random coefficient vector from the oracle's direct
sum, so the least-squares solution is that vector up to the NFFT error; the
tests check the recovered coefficients against it and against a dense
least-squares solve of the oracle's Lambda.

* W = I on Gaussian points (B = 6, FP64, q = 12): relative error <= 1e-7;
* the paper's grid G_N (Section 8) with kappa = 6, N = 20 and the mid-point
  rule weights w_i = (2 kappa / N)^3 e^{-|x_i|^2} as the weights of CGNR
  (B = 8): converges, and in fewer iterations than W = I;
* an FP32 plan (vectors FP32, scalars FP64): relative error <= 1e-4;
* CGNE for fewer samples than coefficients (normal equations of the second
  kind, Section 2): the residual falls below 1e-10 and the result is the
  minimum-norm solution (a dense least-squares solve of the oracle's Lambda).
"""
import numpy as np
import pytest

import oracle
from oracle import stepwise as sw
from tests import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def grid_points(kappa, n):
    """G_N of Section 8: kappa * (2 j / N - 1) per axis, j = 0 .. N - 1."""
    a = kappa * (2.0 * np.arange(n) / n - 1.0)
    x, y, z = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def test_cgnr_recovers_coefficients():
    import paper_1809_10786_amd as sgl

    B = 6
    pts = wl.gaussian_points(20_000, 110)
    fh = wl.coefficients(B, 111)
    y = oracle.direct_forward(B, pts, fh)
    p = sgl.Plan(dev(pts, torch.float64), B, q=12)
    x, info = p.cgnr(dev(y, torch.complex128), maxiter=300, tol=1e-12)
    x = host(x)
    lam = sw.sgl_basis(B, pts)
    ls = np.linalg.lstsq(lam, y, rcond=None)[0]
    say(f"cgnr W=I: {info}, vs truth {rel(x, fh):.3g}, vs dense lstsq {rel(x, ls):.3g}")
    assert rel(x, fh) < 1e-7 and rel(x, ls) < 1e-7
    p.close()


def test_cgnr_midpoint_weights_on_the_grid():
    import paper_1809_10786_amd as sgl

    B, kappa, n = 8, 6.0, 20
    pts = grid_points(kappa, n)
    fh = wl.coefficients(B, 112)
    y = oracle.direct_forward(B, pts, fh)
    rho = 1.0001 * np.linalg.norm(pts, axis=1).max()
    p = sgl.Plan(dev(pts, torch.float64), B, q=12, rho=rho)
    w = (2 * kappa / n) ** 3 * np.exp(-np.sum(pts * pts, axis=1))
    W = dev(w, torch.float64)
    Y = dev(y, torch.complex128)
    # the mid-point rule itself: fhat0 = Lambda^H (w y)
    x0 = p.adjoint(W.to(torch.complex128) * Y)
    say(f"mid-point rule: {rel(host(x0), fh):.3g}")
    xw, iw = p.cgnr(Y, weights=W, x0=x0, maxiter=2000, tol=1e-10)
    xp, ip = p.cgnr(Y, x0=x0, maxiter=2000, tol=1e-10)
    say(f"weighted {iw} -> {rel(host(xw), fh):.3g}; plain {ip} -> {rel(host(xp), fh):.3g}")
    assert rel(host(xw), fh) < 1e-6
    assert iw["iterations"] < ip["iterations"]
    p.close()


def test_cgnr_fp32_plan():
    import paper_1809_10786_amd as sgl

    B = 6
    pts = wl.gaussian_points(20_000, 113)
    pu = pts.astype(np.float32).astype(np.float64)
    fh = wl.coefficients(B, 114)
    y = oracle.direct_forward(B, pu, fh).astype(np.complex64)
    p = sgl.Plan(dev(pu, torch.float32), B, q=6, precision="f32")
    x, info = p.cgnr(dev(y, torch.complex64), maxiter=300, tol=1e-6)
    say(f"cgnr fp32: {info}, vs truth {rel(host(x), fh):.3g}")
    assert rel(host(x), fh) < 1e-4
    p.close()


def test_cgne_minimum_norm_solution():
    import paper_1809_10786_amd as sgl

    B, M = 8, 100  # Nc = 204 > M; cond(Lambda) about 4e3 on these points
    pts = wl.gaussian_points(M, 160)
    fstar = wl.coefficients(B, 161)
    lam = sw.sgl_basis(B, pts)
    y = lam @ fstar
    say(f"cgne B={B} M={M} Nc={lam.shape[1]}")
    p = sgl.Plan(dev(pts, torch.float64), B, q=12)
    x, info = p.cgne(dev(y, torch.complex128), maxiter=5000, tol=1e-11)
    x = host(x)
    xmin = np.linalg.lstsq(lam, y, rcond=None)[0]  # minimum-norm solution
    say(f"  iterations {info['iterations']} residual {info['rel_residual']:.3g} "
        f"against the minimum-norm solution {rel(x, xmin):.3g}")
    assert info["rel_residual"] <= 1e-11
    assert rel(lam @ x, y) < 1e-9
    assert rel(x, xmin) < 1e-6
    p.close()
