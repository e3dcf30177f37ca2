"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-only functions and argument checks behave as
documented.  Nothing here touches a GPU: every sgl_plan call below fails its
host-side validation before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgl.h")


def _lib():
    import paper_1809_10786_amd as sgl

    if not os.path.exists(sgl.LIB_PATH):
        from paper_1809_10786_amd import build

        build.build()
    return sgl


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sgl_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    sgl = _lib()
    L = sgl.lib()
    decl = declared_symbols()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(sgl.SYMBOLS) == decl


def test_host_only_functions():
    sgl = _lib()
    assert sgl.num_coeffs(8) == 204
    assert sgl.num_coeffs(64) == 89440
    assert sgl.num_coeffs(0) == -1
    mu = 0
    for n in range(1, 9):
        for l in range(n):
            for m in range(-l, l + 1):
                assert sgl.coeff_index(n, l, m) == mu
                mu += 1
    assert sgl.coeff_index(2, 2, 0) == -1
    assert sgl.coeff_index(3, 1, 2) == -1
    assert sgl.eta_dims(64) == (256, 128, 128)
    for s in (0, -1, -2, -3, -4, -5):
        assert sgl.status_string(s)
    assert sgl.status_string(-99) == "unknown status"


@pytest.mark.parametrize(
    "B,sigma,q,prec,flags,M",
    [
        (1, 2, 6, 0, 0, 10),       # B < 2
        (300, 2, 6, 0, 0, 10),     # B too large
        (8, 1, 6, 0, 0, 10),       # sigma < 2
        (8, 2, 0, 0, 0, 10),       # q < 1
        (8, 2, 17, 0, 0, 10),      # 2q > sigma * 2B
        (8, 2, 6, 7, 0, 10),       # bad precision
        (8, 2, 6, 0, 1 << 5, 10),  # unknown flag
        (8, 2, 6, 0, 0, 0),        # M < 1
        (8, 2, 6, 0, 0, 1 << 31),  # M too large
    ],
)
def test_plan_rejects_bad_arguments(B, sigma, q, prec, flags, M):
    sgl = _lib()
    L = sgl.lib()
    prm = sgl.SglParams(B, sigma, q, 0.0, prec, flags)
    h = ctypes.c_void_p(123)
    st = L.sgl_plan(ctypes.byref(h), ctypes.byref(prm), M, ctypes.c_void_p(0x1000), None)
    assert st == sgl.SGL_E_INVAL
    assert h.value is None


@pytest.mark.parametrize("B,sigma", [(171, 3), (129, 4), (256, 4)])
def test_plan_rejects_oversized_fft_grids(B, sigma):
    """FFT lengths are sigma n_j or the next even length whose factors are 2, 3
    and 5; grids beyond 2048 x 1024 x 1024 are refused on the host, before any
    device call."""
    sgl = _lib()
    L = sgl.lib()
    prm = sgl.SglParams(B, sigma, 3, 0.0, 0, 0)
    h = ctypes.c_void_p(123)
    st = L.sgl_plan(ctypes.byref(h), ctypes.byref(prm), 10, ctypes.c_void_p(0x1000), None)
    assert st == sgl.SGL_E_UNSUPPORTED
    assert h.value is None


@pytest.mark.parametrize("B", [49, 64])
def test_split16_conversion_refused_above_its_bandwidth(B):
    """The FP16 hi/lo conversion products miss 1e-5 at B = 64: bandwidths above
    SGL_CONV_SPLIT16_MAX_B are refused on the host, before any device call."""
    sgl = _lib()
    L = sgl.lib()
    prm = sgl.SglParams(B, 2, 6, 0.0, 1, sgl.SGL_FLAG_CONV_SPLIT16)
    h = ctypes.c_void_p(123)
    st = L.sgl_plan(ctypes.byref(h), ctypes.byref(prm), 10, ctypes.c_void_p(0x1000), None)
    assert st == sgl.SGL_E_UNSUPPORTED
    assert h.value is None


def test_null_arguments():
    sgl = _lib()
    L = sgl.lib()
    prm = sgl.SglParams(8, 2, 6, 0.0, 0, 0)
    assert L.sgl_plan(None, ctypes.byref(prm), 10, ctypes.c_void_p(0x1000), None) == sgl.SGL_E_INVAL
    h = ctypes.c_void_p()
    assert L.sgl_plan(ctypes.byref(h), None, 10, ctypes.c_void_p(0x1000), None) == sgl.SGL_E_INVAL
    assert L.sgl_plan(ctypes.byref(h), ctypes.byref(prm), 10, None, None) == sgl.SGL_E_INVAL
    nan = sgl.SglParams(8, 2, 6, float("nan"), 0, 0)
    assert L.sgl_plan(ctypes.byref(h), ctypes.byref(nan), 10, ctypes.c_void_p(0x1000), None) == sgl.SGL_E_INVAL
    for name in ("sgl_forward", "sgl_adjoint", "sgl_conv_forward", "sgl_conv_adjoint", "sgl_nfft_forward",
                 "sgl_nfft_adjoint"):
        assert getattr(L, name)(None, ctypes.c_void_p(16), ctypes.c_void_p(32)) == sgl.SGL_E_INVAL
    assert L.sgl_destroy(None) == sgl.SGL_E_INVAL
    info = (ctypes.c_double * 3)()
    assert L.sgl_cgnr(None, ctypes.c_void_p(16), None, ctypes.c_void_p(32), 10, 1e-6, info) == sgl.SGL_E_INVAL
    assert L.sgl_grad_points(None, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48),
                             ctypes.c_void_p(64)) == sgl.SGL_E_INVAL
    v = ctypes.c_void_p(16)
    assert L.sgl_mlp_num_params() == 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    assert L.sgl_point_features(None, v, v) == sgl.SGL_E_INVAL
    assert L.sgl_mlp_forward(None, v, v, v) == sgl.SGL_E_INVAL
    assert L.sgl_mlp_backward(None, v, v, v, v) == sgl.SGL_E_INVAL
    assert L.sgl_mlp_adam(None, v, v, v, v, 1e-3, 0.9, 0.999, 1e-8, 1) == sgl.SGL_E_INVAL
    assert L.sgl_mlp_weights(None, None, v, v) == sgl.SGL_E_INVAL
    assert L.sgl_mlp_weight_grad(None, v, v, v, 1.0, v) == sgl.SGL_E_INVAL
    loss = ctypes.c_double()
    assert L.sgl_mlp_train_step(None, v, v, v, v, v, 1, 1e-3, 1, ctypes.byref(loss)) == sgl.SGL_E_INVAL
    assert L.sgl_batch_create(None, None, 1, None, None, None, None, 1, None) == sgl.SGL_E_INVAL
    b = ctypes.c_void_p(123)
    hs = (ctypes.c_void_p * 2)(16, 32)
    arr = (ctypes.c_void_p * 2)(64, 4096)
    # no plans, n = 0, no direction, a direction with one of its two arrays missing, bad branch count
    assert L.sgl_batch_create(ctypes.byref(b), None, 2, arr, arr, None, None, 1, None) == sgl.SGL_E_INVAL
    assert b.value is None
    assert L.sgl_batch_create(ctypes.byref(b), hs, 0, arr, arr, None, None, 1, None) == sgl.SGL_E_INVAL
    assert L.sgl_batch_create(ctypes.byref(b), hs, 2, None, None, None, None, 1, None) == sgl.SGL_E_INVAL
    assert L.sgl_batch_create(ctypes.byref(b), hs, 2, arr, None, None, None, 1, None) == sgl.SGL_E_INVAL
    assert L.sgl_batch_create(ctypes.byref(b), hs, 2, arr, arr, None, None, 0, None) == sgl.SGL_E_INVAL
    assert L.sgl_batch_create(ctypes.byref(b), hs, 2, arr, arr, None, None, 17, None) == sgl.SGL_E_INVAL
    assert L.sgl_batch_run(None) == sgl.SGL_E_INVAL and L.sgl_batch_destroy(None) == sgl.SGL_E_INVAL
    assert L.sgl_forward_adjoint(None, v, v, v, v) == sgl.SGL_E_INVAL
    assert L.sgl_plan_rho(None, None) == sgl.SGL_E_INVAL
    assert L.sgl_eta_dims(8, None) == sgl.SGL_E_INVAL


def test_product_path_does_not_import_oracle():
    """The library binding never reaches the oracle (test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_1809_10786_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "liboracle" not in text, f
