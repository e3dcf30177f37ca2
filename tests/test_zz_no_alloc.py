"""sgl_mlp_backward_noalloc (the network's parameter gradient with its
per-block partials in the library's fixed device array, for callers that
cannot allocate) against sgl_mlp_backward, through the C ABI.

Two calls in a row, the second on a plan with fewer points (fewer blocks:
partials the first call left in the array beyond the second call's blocks
must not reach the result), each compared with the allocating entry point bit
for bit (same kernels, same summation order) and with the oracle's gradient
(oracle/learn.py, 1e-4 of the largest entry, the network being FP32); plans
above the array's size are refused with SGL_E_UNSUPPORTED.
"""
import numpy as np
import pytest

from oracle import learn as ol
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


def grads(sgl, plan, params, feat, dc):
    """(allocating, no-allocation) gradients of sum_i dc_i c_i."""
    out = []
    for name in ("sgl_mlp_backward", "sgl_mlp_backward_noalloc"):
        g = torch.full((ol.num_params(),), float("nan"), dtype=torch.float32, device="cuda")
        st = getattr(sgl.lib(), name)(plan._h, sgl._ptr(params), sgl._ptr(feat), sgl._ptr(dc), sgl._ptr(g))
        assert st == sgl.SGL_OK, (name, sgl.status_string(st))
        out.append(host(g).astype(np.float64))
    return out


def test_noalloc_backward_equals_allocating_backward():
    import paper_1809_10786_amd as sgl

    rng = np.random.default_rng(500)
    p = rng.uniform(-0.5, 0.5, ol.num_params()).astype(np.float32)
    params = dev(p, torch.float32)
    for M in (250_000, 3_001):
        say(f"no-alloc backward M={M}")
        plan = sgl.Plan(dev(wl.gaussian_points(M, 501), torch.float64), 4)
        feat = (rng.standard_normal((M, 4)) * 2).astype(np.float32)
        dc = rng.standard_normal(M).astype(np.float32)
        F, DC = dev(feat, torch.float32), dev(dc, torch.float32)
        g_alloc, g_noalloc = grads(sgl, plan, params, F, DC)
        assert np.all(np.isfinite(g_noalloc))
        assert np.array_equal(g_alloc, g_noalloc)
        gref = ol.mlp_grad(p.astype(np.float64), feat.astype(np.float64), dc.astype(np.float64))
        err = np.max(np.abs(g_noalloc - gref)) / np.max(np.abs(gref))
        say(f"  bit-equal to sgl_mlp_backward; against the oracle {err:.3g}")
        assert err <= 1e-4
        plan.close()


def test_noalloc_backward_rejects_plans_above_its_size():
    import paper_1809_10786_amd as sgl

    M = sgl.SGL_MLP_NOALLOC_MAX_POINTS + 1
    plan = sgl.Plan(dev(wl.gaussian_points(M, 502), torch.float64), 4)
    F = torch.zeros((M, 4), dtype=torch.float32, device="cuda")
    DC = torch.zeros(M, dtype=torch.float32, device="cuda")
    params = torch.zeros(ol.num_params(), dtype=torch.float32, device="cuda")
    g = torch.zeros(ol.num_params(), dtype=torch.float32, device="cuda")
    st = sgl.lib().sgl_mlp_backward_noalloc(plan._h, sgl._ptr(params), sgl._ptr(F), sgl._ptr(DC), sgl._ptr(g))
    assert st == sgl.SGL_E_UNSUPPORTED
    assert sgl.lib().sgl_mlp_backward_noalloc(plan._h, None, sgl._ptr(F), sgl._ptr(DC), sgl._ptr(g)) == sgl.SGL_E_INVAL
    plan.close()
