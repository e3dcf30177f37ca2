"""Seeded synthetic inputs shared by the oracle-side and GPU-side tests and by
bench.py.  Holds no arithmetic of the transform itself: only random numbers
with the shapes and distributions of the workloads.

The paper measures on seeded random data only (uniform coefficients, points
uniform in balls, Section 8); the workloads below keep that structure at the
sizes used for parity tests and for the throughput measurement.
"""
import numpy as np


def num_coeffs(B):
    return B * (B + 1) * (2 * B + 1) // 6


def degree_n(B):
    """The first index n of every coefficient, in coefficient order (n outer)."""
    return np.concatenate([np.full(n * n, n, dtype=np.int64) for n in range(1, B + 1)])


def coefficients(B, seed, decay=1.5):
    """Re, Im iid N(0,1), scaled by n^-decay."""
    rng = np.random.default_rng(seed)
    nc = num_coeffs(B)
    c = rng.standard_normal(nc) + 1j * rng.standard_normal(nc)
    return c * degree_n(B).astype(np.float64) ** (-decay)


def coefficients_uniform(B, seed):
    """Re, Im iid U[-1, 1] (the coefficient distribution of Section 8)."""
    rng = np.random.default_rng(seed)
    nc = num_coeffs(B)
    return rng.uniform(-1, 1, nc) + 1j * rng.uniform(-1, 1, nc)


def gaussian_points(M, seed):
    """Points iid N(0, I/2): density proportional to exp(-r^2), the weight of H."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((M, 3)) * np.sqrt(0.5)


def ball_points(M, radius, seed):
    """Points uniform in the ball of the given radius (Section 8)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((M, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.uniform(0, 1, M) ** (1.0 / 3.0)
    return d * r[:, None]


def ball_points_centered(M, radius, seed):
    """Points in the ball of the given radius with radius * U^(1/2) as their
    distance from the origin: point density falling as 1/r towards the rim."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((M, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * (radius * rng.uniform(0, 1, M) ** 0.5)[:, None]


def mixed_points(M, seed, frac_ball=0.1, radius=4.0):
    """(1 - frac_ball) M Gaussian points plus frac_ball M uniform in a ball."""
    mb = int(round(M * frac_ball))
    g = gaussian_points(M - mb, seed)
    b = ball_points(mb, radius, seed + 1)
    return np.concatenate([g, b], axis=0)


def mixture_points(M, seed, k=3, diag_lo=0.3, diag_hi=2.0):
    """Anisotropic Gaussian mixture: k components with equal weights, means
    iid U[-1, 1]^3 and diagonal covariances with entries iid U[diag_lo, diag_hi]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (k, 3))
    cov = rng.uniform(diag_lo, diag_hi, (k, 3))
    comp = rng.integers(0, k, M)
    return means[comp] + rng.standard_normal((M, 3)) * np.sqrt(cov[comp])


def clustered_points(M, seed, k=8):
    """Gaussian mixture of k isotropic clusters, weights ~ Dirichlet(1), means
    iid N(0, I/2), cluster variances iid U[0.02, 0.2]."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(k))
    means = rng.standard_normal((k, 3)) * np.sqrt(0.5)
    var = rng.uniform(0.02, 0.2, k)
    comp = rng.choice(k, M, p=w)
    return means[comp] + rng.standard_normal((M, 3)) * np.sqrt(var[comp])[:, None]


def samples(M, seed):
    """Adjoint input y: iid complex N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(M) + 1j * rng.standard_normal(M)


# Workloads: name -> (B, M, point generator, coefficient decay, sigma, q, precision)
WORKLOADS = {
    # FP64 forward + adjoint at B=8, M=1e4 Gaussian points, n^-2 decay; q = 16 as in Section 8.
    "b8_m1e4_f64": dict(B=8, M=10_000, points="gaussian", decay=2.0, sigma=2, q=16, prec="f64"),
    # B=32, M=1e6 (0.9e6 Gaussian + 0.1e6 uniform in the ball r <= 4), n^-1.5, q=6.
    "b32_m1e6_f64": dict(B=32, M=1_000_000, points="mixed", decay=1.5, sigma=2, q=6, prec="f64"),
    "b32_m1e6_f32": dict(B=32, M=1_000_000, points="mixed", decay=1.5, sigma=2, q=6, prec="f32"),
    # Throughput workload: B=64, M=4e6 Gaussian points, n^-1.5, FP32, q=6.
    "b64_m4e6_f32": dict(B=64, M=4_000_000, points="gaussian", decay=1.5, sigma=2, q=6, prec="f32"),
    "b64_m4e6_f64": dict(B=64, M=4_000_000, points="gaussian", decay=1.5, sigma=2, q=6, prec="f64"),
    # The same at the high-accuracy cutoff q = 14 (Theorem 2.7; ~1e-10 and below in FP64).
    "b64_m4e6_f64_q14": dict(B=64, M=4_000_000, points="gaussian", decay=1.5, sigma=2, q=14, prec="f64"),
    # Inverse transform: B=32, M=3e5 FP64 points in eight clusters (Dirichlet(1) weights), n^-1.5, q=6.
    "b32_m3e5_clustered_f64": dict(B=32, M=300_000, points="clustered8", decay=1.5, sigma=2, q=6, prec="f64"),
    # Inverse transform where a normal residual of 1e-6 is reachable: B=12, M=2e4 FP64 points
    # covering the ball of radius 5, density falling as 1/r, n^-1.5, q=8.
    "b12_m2e4_centered5_f64": dict(B=12, M=20_000, points="centered5", decay=1.5, sigma=2, q=8, prec="f64"),
    # B=48, M=2e6 FP32 points from a 3-component anisotropic Gaussian mixture, n^-1.5, q=6.
    "b48_m2e6_f32": dict(B=48, M=2_000_000, points="aniso3", decay=1.5, sigma=2, q=6, prec="f32"),
}


def make_points(kind, M, seed):
    if kind == "gaussian":
        return gaussian_points(M, seed)
    if kind == "mixed":
        return mixed_points(M, seed)
    if kind == "aniso3":
        return mixture_points(M, seed)
    if kind == "clustered8":
        return clustered_points(M, seed)
    if kind.startswith("centered"):
        return ball_points_centered(M, float(kind[8:]), seed)
    if kind.startswith("ball"):
        return ball_points(M, float(kind[4:]), seed)
    raise ValueError(kind)


def workload(name, seed=0, M=None):
    w = dict(WORKLOADS[name])
    if M is not None:
        w["M"] = M
    pts = make_points(w["points"], w["M"], seed)
    fhat = coefficients(w["B"], seed + 100, w["decay"])
    y = samples(w["M"], seed + 200)
    return w, pts, fhat, y


def batch_specs(n=64, seed=0, b_lo=16, b_hi=64, m_lo=1e5, m_hi=2e6):
    """(B, M) of a batch: B uniform in [b_lo, b_hi], M log-uniform in [m_lo, m_hi]."""
    rng = np.random.default_rng(seed)
    bs = list(range(b_lo, b_hi + 1))
    B = rng.choice(bs, n)
    M = np.exp(rng.uniform(np.log(m_lo), np.log(m_hi), n)).astype(np.int64)
    return [(int(b), int(m)) for b, m in zip(B, M)]
