"""GPU parity at the full workload sizes and on the FP32 matrix-core path.

* the throughput workload (B=64, M=4e6, FP32 and FP64) in the launch
  configuration the benchmark times, the B=32, M=1e6 mixed point set and the
  B=48, M=2e6 anisotropic mixture, against the direct sum (Def. 1.3):
  - the forward element by element on 2^16 seeded sampled points;
  - the adjoint of DENSE samples (all M points, iid complex N(0, 1)) element
    by element against the direct adjoint Lambda^H y (every one of the Nc
    coefficients), which exercises every chunk, the running exponent of the
    FP32 spread, and the full-size fold;
  - two adjoint runs on the same input equal bit for bit (no atomics, fixed
    summation order);
  - the adjoint identity <Lambda fhat, y> = <fhat, Lambda^H y> with every
    point;
* the NFFT stage on the matrix-core gather and spread (tiles of 8^3 cells;
  FP16 hi/lo products for FP32 plans, FP64 products for FP64 plans) against
  the FP64 stepwise Gaussian NFFT: several tiles with ragged point counts,
  one tile holding more than one chunk of points, all-zero input and inputs
  scaled by 2^+-80.
Tolerances: FP32 1e-5 relative (l2 and max), FP64 at q=6 2e-6 (the Gaussian
window's truncation error, Theorem 2.7), identity 2e-6 (FP32) / 1e-12 (FP64)
relative to |y| |Lambda fhat|.
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def relinf(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def as_used(x, prec):
    """Inputs exactly as the library sees them."""
    if prec == "f64":
        return x
    if np.iscomplexobj(x):
        return x.astype(np.complex64).astype(np.complex128)
    return x.astype(np.float32).astype(np.float64)


def check_workload(name, prec, seed, nsample, tol, idtol):
    import paper_1809_10786_amd as sgl

    w, pts, fh, y = wl.workload(name, seed=seed)
    B, M = w["B"], len(pts)
    say(f"full {name} {prec} B={B} M={M} q={w['q']}")
    rdt, cdt = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    p = sgl.Plan(dev(pts, rdt), B, sigma=w["sigma"], q=w["q"], precision=prec)
    if w["q"] <= 6:
        # the matrix-core gather and spread: FP16 hi/lo for FP32 plans, FP64 otherwise
        assert p.info()["gather_mode"] == (2 if prec == "f32" else 3)
    pu, fhu, yu = as_used(pts, prec), as_used(fh, prec), as_used(y, prec)
    f = host(p.forward(dev(fh, cdt)))
    idx = np.sort(np.random.default_rng(seed + 7).choice(M, min(nsample, M), replace=False))
    f0 = oracle.direct_forward(B, pu[idx], fhu)
    say(f"  forward ({len(idx)} points) rel l2 {rel(f[idx], f0):.3g} max {relinf(f[idx], f0):.3g}")
    assert rel(f[idx], f0) < tol and relinf(f[idx], f0) < tol
    # dense adjoint: every point carries a sample
    dy = dev(y, cdt)
    g = host(p.adjoint(dy))
    g2 = host(p.adjoint(dy))
    assert np.array_equal(g, g2), "two adjoint runs differ"
    say(f"  adjoint of dense y: direct sum over {M} points ...")
    g0 = oracle.direct_adjoint(B, pu, yu)
    say(f"  adjoint rel l2 {rel(g, g0):.3g} max {relinf(g, g0):.3g}")
    assert rel(g, g0) < tol and relinf(g, g0) < tol
    # adjoint identity with every point
    lhs, rhs = np.vdot(yu, f), np.vdot(g, fhu)
    say(f"  identity {abs(lhs - rhs) / (np.linalg.norm(yu) * np.linalg.norm(f)):.3g}")
    assert abs(lhs - rhs) < idtol * np.linalg.norm(yu) * np.linalg.norm(f)
    p.close()


NFWD = 1 << 16


def test_b64_m4e6_f32_launch_configuration():
    check_workload("b64_m4e6_f32", "f32", 11, NFWD, 1e-5, 2e-6)


def test_b64_m4e6_f64():
    check_workload("b64_m4e6_f64", "f64", 12, NFWD, 2e-6, 1e-12)


def test_b64_m4e6_f64_q14():
    """The high-accuracy cutoff q = 14 (cell-owned scatter, slab-streamed gather)."""
    check_workload("b64_m4e6_f64_q14", "f64", 17, NFWD, 1e-10, 1e-12)


@pytest.mark.parametrize("prec,tol,idtol", [("f32", 1e-5, 2e-6), ("f64", 2e-6, 1e-12)])
def test_b32_m1e6_mixed(prec, tol, idtol):
    check_workload("b32_m1e6_" + prec, prec, 13, NFWD, tol, idtol)


def test_b48_m2e6_anisotropic_mixture_f32():
    check_workload("b48_m2e6_f32", "f32", 14, NFWD, 1e-5, 2e-6)


# ------------------------------------------------------------ FP32 NFFT stage


def stage_points(seed):
    """2000 Gaussian points plus 4500 points packed into one tile (three
    chunks: the plan caps a chunk at 2048 points), at rho = 1.1 max r."""
    rng = np.random.default_rng(seed)
    a = wl.gaussian_points(2000, seed)
    c = np.array([0.35, -0.2, 0.5]) + 1e-3 * rng.standard_normal((4500, 3))
    return np.concatenate([a, c], axis=0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("B", [8, 12])
def test_nfft_stage_matrix_cores(B, prec):
    """The matrix-core gather and spread (FP16 hi/lo for FP32 plans at 1e-5,
    FP64 for FP64 plans at 1e-11) against the stepwise NFFT."""
    import paper_1809_10786_amd as sgl

    q = 6
    pts = stage_points(50 + B)
    rho = 1.1 * np.linalg.norm(pts, axis=1).max()
    say(f"{prec} nfft stage B={B} M={len(pts)}")
    rdt, cdt = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-11 if prec == "f64" else 1e-5
    p = sgl.Plan(dev(pts, rdt), B, q=q, rho=rho, precision=prec)
    info = p.info()
    assert info["gather_mode"] == (3 if prec == "f64" else 2) and (info["L0"], info["L1"], info["L2"]) == (8, 8, 8)
    t = sw.x_tilde(as_used(pts, prec), p.rho)
    rng = np.random.default_rng(60 + B)
    eta = as_used(rng.standard_normal(p.eta_shape) + 1j * rng.standard_normal(p.eta_shape), prec)
    y = as_used(wl.samples(len(pts), 70 + B), prec)
    f0 = sw.nfft(eta, t, 2, q)
    e0 = sw.nfft_adjoint(y, t, p.eta_shape, 2, q).reshape(-1)
    for scale in (1.0, 2.0 ** 80, 2.0 ** -80):
        f = host(p.nfft_forward(dev(eta * scale, cdt))) / scale
        e = host(p.nfft_adjoint(dev(y * scale, cdt))).reshape(-1) / scale
        say(f"  scale {scale:.3g}: forward {rel(f, f0):.3g} / {relinf(f, f0):.3g}, "
            f"adjoint {rel(e, e0):.3g} / {relinf(e, e0):.3g}")
        assert rel(f, f0) < tol and relinf(f, f0) < tol
        assert rel(e, e0) < tol and relinf(e, e0) < tol
    z = host(p.nfft_forward(torch.zeros(p.eta_shape, dtype=cdt, device="cuda")))
    assert not np.any(z)
    z = host(p.nfft_adjoint(torch.zeros(len(pts), dtype=cdt, device="cuda")))
    assert not np.any(z)
    p.close()
