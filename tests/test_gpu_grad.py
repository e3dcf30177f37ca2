"""Differentiation (gradient with respect to coefficients and point positions).

* sgl_grad_points against the oracle's analytic gradient d H_nlm / d x
  (oracle.stepwise.sgl_basis_grad, itself pinned to central differences of the
  direct sum and to closed forms): FP64 at q = 10 (1e-7 relative to the
  largest component), FP32 at q = 6 (1e-4);
* against central differences of the GPU forward itself (new plans at x +- h e_c
  with rho held fixed): FP64, h = 1e-5, 1e-6;
* the torch.autograd.Function: gradients of a least-squares loss against a
  dense-matrix reference built from the oracle (fhat) and the analytic oracle
  gradient (points), FP64;
* the differentiation workload's shape (B = 48, 2e6 FP32 points from the
  anisotropic mixture): sampled point gradients against the oracle, 1e-4.
"""
import numpy as np
import pytest

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
    return t.cpu().numpy()


def oracle_grad(B, pts, fh, g):
    """Re(conj(g_i) d f_i / d x_ic) from the analytic oracle gradient."""
    df = sw.forward_grad(B, pts, fh)  # (M, 3) complex
    return np.real(np.conj(g)[:, None] * df)


def err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("B,prec,q,tol", [(8, "f64", 10, 1e-7), (16, "f64", 10, 1e-7), (16, "f32", 6, 1e-4)])
def test_grad_points_against_oracle(B, prec, q, tol):
    import paper_1809_10786_amd as sgl

    pts = wl.gaussian_points(400, 90 + B)
    rdt, cdt = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    pu = pts.astype(np.float32).astype(np.float64) if prec == "f32" else pts
    rho = 1.05 * np.linalg.norm(pu, axis=1).max()
    fh = wl.coefficients(B, 91 + B)
    g = wl.samples(len(pts), 92 + B)
    if prec == "f32":
        fh = fh.astype(np.complex64).astype(np.complex128)
        g = g.astype(np.complex64).astype(np.complex128)
    P = dev(pu, rdt)
    p = sgl.Plan(P, B, q=q, rho=rho, precision=prec)
    gr = host(p.grad_points(dev(fh, cdt), P, dev(g, cdt))).astype(np.float64)
    g0 = oracle_grad(B, pu, fh, g)
    say(f"grad B={B} {prec} q={q}: {err(gr, g0):.3g}")
    assert err(gr, g0) < tol
    p.close()


def test_grad_points_against_central_differences():
    import paper_1809_10786_amd as sgl

    B, q, h = 12, 8, 1e-5
    pts = wl.mixed_points(1500, 93)
    rho = 1.05 * np.linalg.norm(pts, axis=1).max()
    fh = wl.coefficients(B, 94)
    g = wl.samples(len(pts), 95)
    P = dev(pts, torch.float64)
    p = sgl.Plan(P, B, q=q, rho=rho)
    gr = host(p.grad_points(dev(fh, torch.complex128), P, dev(g, torch.complex128)))
    sel = [3, 500, 1499]
    worst = 0.0
    for c in range(3):
        fd = np.zeros(len(pts))
        for s in (+1, -1):
            q_pts = pts.copy()
            q_pts[sel, c] += s * h
            pp = sgl.Plan(dev(q_pts, torch.float64), B, q=q, rho=rho)
            f = host(pp.forward(dev(fh, torch.complex128)))
            fd = fd + s * np.real(np.conj(g) * f) / (2 * h)
            pp.close()
        for i in sel:
            worst = max(worst, abs(gr[i, c] - fd[i]) / np.abs(gr[sel]).max())
    say(f"central differences: {worst:.3g}")
    assert worst < 1e-6
    p.close()


def test_autograd_function_least_squares():
    import paper_1809_10786_amd as sgl

    B = 6
    pts = wl.gaussian_points(300, 96)
    rho = 1.05 * np.linalg.norm(pts, axis=1).max()
    fh = wl.coefficients(B, 97)
    y = wl.samples(len(pts), 98)
    P = dev(pts, torch.float64).requires_grad_(True)
    plan = sgl.Plan(P.detach(), B, q=10, rho=rho)
    F = dev(fh, torch.complex128).requires_grad_(True)
    f = sgl.transform(F, P, plan)
    loss = (f - dev(y, torch.complex128)).abs().pow(2).sum()
    loss.backward()
    # reference: dense Lambda from the oracle, autograd on the CPU
    Lam = torch.from_numpy(sw.sgl_basis(B, pts))
    Fr = torch.from_numpy(fh).requires_grad_(True)
    fr = Lam @ Fr
    hook = {}
    fr.register_hook(lambda gg: hook.setdefault("g", gg))
    ((fr - torch.from_numpy(y)).abs().pow(2).sum()).backward()
    gf = F.grad.cpu().numpy()
    say(f"autograd fhat: {err(gf, Fr.grad.numpy()):.3g}")
    assert err(gf, Fr.grad.numpy()) < 1e-8
    gx0 = oracle_grad(B, pts, fh, hook["g"].numpy())
    say(f"autograd points: {err(P.grad.cpu().numpy(), gx0):.3g}")
    assert err(P.grad.cpu().numpy(), gx0) < 1e-7
    plan.close()


def test_grad_points_differentiation_workload_shape():
    """B = 48, 2e6 FP32 points from the anisotropic mixture (q = 6)."""
    import paper_1809_10786_amd as sgl

    w, pts, fh, y = wl.workload("b48_m2e6_f32", seed=15)
    B = w["B"]
    pu = pts.astype(np.float32).astype(np.float64)
    rho = 1.0001 * np.linalg.norm(pu, axis=1).max()
    fhu = fh.astype(np.complex64).astype(np.complex128)
    yu = y.astype(np.complex64).astype(np.complex128)
    P = dev(pu, torch.float32)
    p = sgl.Plan(P, B, q=6, rho=rho, precision="f32")
    gr = host(p.grad_points(dev(fhu, torch.complex64), P, dev(yu, torch.complex64))).astype(np.float64)
    idx = np.sort(np.random.default_rng(16).choice(len(pts), 60, replace=False))
    g0 = oracle_grad(B, pu[idx], fhu, yu[idx])
    say(f"grad B=48 M=2e6 f32 (60 sampled points): {err(gr[idx], g0):.3g}")
    assert np.all(np.isfinite(gr[idx]))
    assert err(gr[idx], g0) < 1e-4
    p.close()


@pytest.mark.parametrize("B,prec,q,tol", [(12, "f64", 10, 1e-7), (12, "f32", 6, 1e-4)])
def test_grad_points_default_rho_outermost_point(B, prec, q, tol):
    """A plan with the default rho = max |x| (eq. nfsglft_rho) puts the outermost
    point at x~_0 = 0, where the radial chain rule takes its limit through the
    second window derivative: every gradient is finite, and the outermost
    point's own gradient matches the oracle's analytic one."""
    import paper_1809_10786_amd as sgl

    pts = wl.gaussian_points(800, 120 + B)
    rdt, cdt = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    pu = pts.astype(np.float32).astype(np.float64) if prec == "f32" else pts
    fh = wl.coefficients(B, 121 + B)
    g = wl.samples(len(pts), 122 + B)
    if prec == "f32":
        fh = fh.astype(np.complex64).astype(np.complex128)
        g = g.astype(np.complex64).astype(np.complex128)
    P = dev(pu, rdt)
    p = sgl.Plan(P, B, q=q, precision=prec)
    k = int(np.argmax(np.linalg.norm(pu, axis=1)))
    assert abs(p.rho - np.linalg.norm(pu[k])) <= 1e-14 * p.rho
    gr = host(p.grad_points(dev(fh, cdt), P, dev(g, cdt))).astype(np.float64)
    assert np.all(np.isfinite(gr))
    g0 = oracle_grad(B, pu, fh, g)
    ek = float(np.abs(gr[k] - g0[k]).max() / np.abs(g0[k]).max())
    say(f"grad default rho B={B} {prec}: all points {err(gr, g0):.3g}, outermost point {ek:.3g}")
    assert err(gr, g0) < tol
    assert ek < 10 * tol
    p.close()
