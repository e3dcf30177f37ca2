"""ORACLE -- test infrastructure only (see ``oracle/__init__.py``).

Learned density-compensation weights for the inverse transform, written out
from their definitions in plain numpy at float64.

The inverse NFSGLFT (Section 8) recovers fhat from samples y = Lambda fhat by
CGNR; weights w_i that make Lambda^H W Lambda close to the identity speed it up.
The SGL functions are orthonormal for the weight e^{-r^2} (Section 1), so a
quadrature with nodes x_i has weights about e^{-|x_i|^2} times the volume each
node stands for, the mid-point rule of Section 8 being the case of a Cartesian
grid.  For scattered nodes that volume is about 1 / (M density); the weights
here are

    w_i = exp(c_i - d_i - |x_i|^2) / M,   c = MLP(features_i),

with d_i the log density of a histogram.  The pieces:

* ``features``: for cells of edge 2 rho / n, n = 64, 32, 16, over [-rho, rho]^3,
  the log of (count of points in x_i's cell) / (M h^3), and |x_i|^2 / rho^2.
  Cell index floor((v + rho) / (2 rho) n), clamped to [0, n - 1].
* ``mlp``: 4 -> 64 -> 64 -> 1 with tanh hidden layers; parameters packed as
  W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3.
* ``mlp_grad``: the gradient of sum_i dc_i c_i with respect to the packed
  parameters, by the chain rule layer by layer.
* ``adam``: one step of Adam (Kingma & Ba, 2015) with bias correction.
* ``loss_and_dc``: for coefficient vectors fhat_b, L = mean_b |e_b|^2 / |fhat_b|^2
  with e_b = Lambda^H (w y_b) - fhat_b and y_b = Lambda fhat_b, and its gradient
  with respect to c: dL/dw_i = 2 Re(y_i conj((Lambda e)_i)) / (nb |fhat_b|^2),
  dw_i/dc_i = w_i.  Lambda and Lambda^H are the direct sums of the C oracle.

Pins (tests/test_oracle_learn.py): lattice points with a known count per cell
(closed-form densities), the network against torch.nn layers in float64, the
parameter gradient against central differences of ``mlp``, Adam against
torch.optim.Adam, and dL/dc against central differences of the loss.
"""
import numpy as np

H, F = 64, 4
GRIDS = (64, 32, 16)


def num_params():
    return H * F + H + H * H + H + H + 1


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]])


def cell_index(points, rho, n):
    """Linear cell index (ix n + iy) n + iz of each point."""
    c = np.floor((points + rho) / (2.0 * rho) * n).astype(np.int64)
    c = np.clip(c, 0, n - 1)
    return (c[:, 0] * n + c[:, 1]) * n + c[:, 2]


def features(points, rho):
    """(M, 4) features: log densities at three cell sizes and |x|^2 / rho^2."""
    points = np.asarray(points, dtype=np.float64)
    M = points.shape[0]
    out = np.empty((M, F))
    for s, n in enumerate(GRIDS):
        key = cell_index(points, rho, n)
        counts = np.bincount(key, minlength=n ** 3)[key]
        h = 2.0 * rho / n
        out[:, s] = np.log(counts / (M * h ** 3))
    out[:, 3] = np.sum(points * points, axis=1) / (rho * rho)
    return out


def mlp(params, feat):
    """c_i = W3 . tanh(W2 tanh(W1 x_i + b1) + b2) + b3."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    h1 = np.tanh(feat @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3 + b3


def mlp_grad(params, feat, dc):
    """Gradient of sum_i dc_i c_i with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    h1 = np.tanh(feat @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    d2 = (dc[:, None] * W3[None, :]) * (1.0 - h2 * h2)   # d/d(pre-activation 2)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)                      # d/d(pre-activation 1)
    return pack(d1.T @ feat, d1.sum(0), d2.T @ h1, d2.sum(0), h2.T @ dc, dc.sum())


def adam(params, grad, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def weights(c, feat, rho):
    """w_i = exp(c_i - d_i - |x_i|^2) / M with d_i the middle-scale log density."""
    M = feat.shape[0]
    return np.exp(c - feat[:, 1] - rho * rho * feat[:, 3]) / M


def loss_and_dc(fwd, adj, w, fhats):
    """Loss mean_b |Lambda^H (w Lambda fhat_b) - fhat_b|^2 / |fhat_b|^2 and dL/dc.

    fwd(fhat) -> Lambda fhat and adj(y) -> Lambda^H y are the transforms."""
    nb = len(fhats)
    L, dc = 0.0, np.zeros_like(w)
    for fh in fhats:
        y = fwd(fh)
        e = adj(w * y) - fh
        nf = np.vdot(fh, fh).real
        L += np.vdot(e, e).real / nf / nb
        g = fwd(e)
        dc += 2.0 * np.real(y * np.conj(g)) * w / (nb * nf)
    return L, dc
