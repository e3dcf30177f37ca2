"""Fast SGL Fourier transform for scattered data (NFSGLFT) on MI355X.

Thin ctypes binding over the C-ABI library ``libsgl.so`` (include/sgl.h).
Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  There
is no fallback -- if the library is missing, importing the binding raises.
"""
import ctypes
import functools
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgl.so")

SGL_OK, SGL_E_INVAL, SGL_E_RANGE, SGL_E_NOMEM, SGL_E_DEVICE, SGL_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SGL_F64, SGL_F32 = 0, 1
SGL_FLAG_EXACT_NDFT = 1
SGL_FLAG_CONV_SPLIT16 = 2

# Every symbol include/sgl.h declares.
SYMBOLS = (
    "sgl_num_coeffs", "sgl_coeff_index", "sgl_eta_dims", "sgl_plan", "sgl_forward", "sgl_adjoint",
    "sgl_conv_forward", "sgl_conv_adjoint", "sgl_nfft_forward", "sgl_nfft_adjoint", "sgl_plan_rho",
    "sgl_plan_info", "sgl_plan_profile", "sgl_plan_stage_times", "sgl_destroy", "sgl_status_string",
    "sgl_last_error", "sgl_grad_points", "sgl_cgnr", "sgl_mlp_num_params", "sgl_point_features",
    "sgl_mlp_forward", "sgl_mlp_backward", "sgl_mlp_adam", "sgl_mlp_weights", "sgl_mlp_weight_grad",
    "sgl_mlp_train_step", "sgl_batch_create", "sgl_batch_run", "sgl_batch_destroy", "sgl_forward_adjoint",
    "sgl_mlp_backward_noalloc", "sgl_cgne",
)
SGL_MLP_NOALLOC_MAX_POINTS = 327680

STAGES = ("conv_radial", "conv_polar", "fft_A", "fft_B", "fft_C", "gather", "scatter", "fft_Ch", "fft_Bh",
          "fft_Ah", "conv_polar_adj", "conv_radial_adj", "ndft", "ndft_adj", "fold")


class SglParams(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("sigma", ctypes.c_int32), ("q", ctypes.c_int32),
                ("rho", ctypes.c_double), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class SglError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        detail = ""
        if status in (SGL_E_DEVICE, SGL_E_NOMEM):
            detail = f" [{lib().sgl_last_error().decode()}]"
        super().__init__(f"{what}: {status_string(status)} ({status}){detail}")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1809_10786_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sgl_num_coeffs.argtypes, L.sgl_num_coeffs.restype = [i32], i64
        L.sgl_coeff_index.argtypes, L.sgl_coeff_index.restype = [i32, i32, i32], i64
        L.sgl_eta_dims.argtypes, L.sgl_eta_dims.restype = [i32, ctypes.POINTER(i32)], ctypes.c_int
        L.sgl_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SglParams), i64, vp, vp]
        L.sgl_plan.restype = ctypes.c_int
        for name in ("sgl_forward", "sgl_adjoint", "sgl_conv_forward", "sgl_conv_adjoint",
                     "sgl_nfft_forward", "sgl_nfft_adjoint"):
            fn = getattr(L, name)
            fn.argtypes, fn.restype = [vp, vp, vp], ctypes.c_int
        L.sgl_plan_rho.argtypes, L.sgl_plan_rho.restype = [vp, ctypes.POINTER(ctypes.c_double)], ctypes.c_int
        L.sgl_plan_info.argtypes, L.sgl_plan_info.restype = [vp, ctypes.POINTER(i64)], ctypes.c_int
        L.sgl_plan_profile.argtypes, L.sgl_plan_profile.restype = [vp, i32], ctypes.c_int
        L.sgl_plan_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]
        L.sgl_plan_stage_times.restype = ctypes.c_int
        L.sgl_destroy.argtypes, L.sgl_destroy.restype = [vp], ctypes.c_int
        L.sgl_status_string.argtypes, L.sgl_status_string.restype = [ctypes.c_int], ctypes.c_char_p
        L.sgl_last_error.argtypes, L.sgl_last_error.restype = [], ctypes.c_char_p
        L.sgl_grad_points.argtypes, L.sgl_grad_points.restype = [vp, vp, vp, vp, vp], ctypes.c_int
        L.sgl_forward_adjoint.argtypes, L.sgl_forward_adjoint.restype = [vp, vp, vp, vp, vp], ctypes.c_int
        L.sgl_cgnr.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.sgl_cgne.argtypes = [vp, vp, vp, i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.sgl_cgne.restype = ctypes.c_int
        f32, f64 = ctypes.c_float, ctypes.c_double
        L.sgl_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
        L.sgl_batch_create.restype = ctypes.c_int
        for name in ("sgl_batch_run", "sgl_batch_destroy"):
            fn = getattr(L, name)
            fn.argtypes, fn.restype = [vp], ctypes.c_int
        L.sgl_mlp_num_params.argtypes, L.sgl_mlp_num_params.restype = [], i32
        for name, args in (("sgl_point_features", [vp, vp, vp]), ("sgl_mlp_forward", [vp, vp, vp, vp]),
                           ("sgl_mlp_backward", [vp, vp, vp, vp, vp]),
                           ("sgl_mlp_backward_noalloc", [vp, vp, vp, vp, vp]),
                           ("sgl_mlp_adam", [vp, vp, vp, vp, vp, f32, f32, f32, f32, i32]),
                           ("sgl_mlp_weights", [vp, vp, vp, vp]), ("sgl_mlp_weight_grad", [vp, vp, vp, vp, f64, vp]),
                           ("sgl_mlp_train_step", [vp, vp, vp, vp, vp, vp, i32, f32, i32, ctypes.POINTER(f64)])):
            fn = getattr(L, name)
            fn.argtypes, fn.restype = args, ctypes.c_int
        L.sgl_cgnr.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s):
    return lib().sgl_status_string(s).decode()


def _check(st, what):
    if st != SGL_OK:
        raise SglError(st, what)


def num_coeffs(B):
    return int(lib().sgl_num_coeffs(B))


def coeff_index(n, l, m):
    return int(lib().sgl_coeff_index(n, l, m))


def eta_dims(B):
    d = (ctypes.c_int32 * 3)()
    _check(lib().sgl_eta_dims(B, d), "sgl_eta_dims")
    return tuple(d)


class Plan:
    """NFSGLFT plan for fixed points on the current CUDA (HIP) device.

    points    : torch tensor (M, 3), float64 for precision "f64", float32 for "f32", on the GPU
    B         : bandwidth; sigma, q: NFFT oversampling and cutoff; rho <= 0 picks max |x_i|
    exact_ndft: evaluate the trigonometric polynomial exactly (test mode)
    conv_split16: conversion products on the FP16 matrix cores with hi/lo split operands
    """

    def __init__(self, points, B, sigma=2, q=6, rho=0.0, precision="f64", exact_ndft=False, conv_split16=False,
                 stream=None):
        import torch

        self._torch = torch
        if precision not in ("f64", "f32"):
            raise ValueError("precision must be 'f64' or 'f32'")
        self.precision = precision
        self.real_dtype = torch.float64 if precision == "f64" else torch.float32
        self.complex_dtype = torch.complex128 if precision == "f64" else torch.complex64
        if not points.is_cuda or points.dtype != self.real_dtype or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError(f"points must be a CUDA tensor (M, 3) of {self.real_dtype}")
        points = points.contiguous()
        self.B, self.M = int(B), int(points.shape[0])
        self.device = points.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        prm = SglParams(self.B, int(sigma), int(q), float(rho), SGL_F64 if precision == "f64" else SGL_F32,
                        (SGL_FLAG_EXACT_NDFT if exact_ndft else 0) | (SGL_FLAG_CONV_SPLIT16 if conv_split16 else 0))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().sgl_plan(ctypes.byref(h), ctypes.byref(prm), self.M, ctypes.c_void_p(points.data_ptr()),
                                ctypes.c_void_p(self.stream.cuda_stream))
        _check(st, "sgl_plan")
        self._h = h
        self.nc = num_coeffs(self.B)
        self.eta_shape = eta_dims(self.B)

    # -- properties --------------------------------------------------------
    @property
    def rho(self):
        r = ctypes.c_double()
        _check(lib().sgl_plan_rho(self._h, ctypes.byref(r)), "sgl_plan_rho")
        return r.value

    def info(self):
        v = (ctypes.c_int64 * 12)()
        _check(lib().sgl_plan_info(self._h, v), "sgl_plan_info")
        keys = ("M", "N0", "N1", "N2", "E0", "E1", "E2", "L0", "L1", "L2", "bytes", "gather_mode")
        return dict(zip(keys, list(v)))

    def profile(self, enable=True):
        """Per-stage HIP-event timing of every launch on the plan's stream."""
        _check(lib().sgl_plan_profile(self._h, 1 if enable else 0), "sgl_plan_profile")

    def stage_times(self, reset=True):
        """{stage: (total ms, launches)} since the last reset (waits for the stream)."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(lib().sgl_plan_stage_times(self._h, ms, cnt, 1 if reset else 0), "sgl_plan_stage_times")
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    # -- helpers -------------------------------------------------------------
    def _in(self, x, n, what):
        if not x.is_cuda or x.dtype != self.complex_dtype or x.numel() != n:
            raise ValueError(f"{what} must be a CUDA {self.complex_dtype} tensor with {n} elements")
        return x.contiguous()

    def _out(self, n, out):
        if out is None:
            return self._torch.empty(n, dtype=self.complex_dtype, device=self.device)
        if out.dtype != self.complex_dtype or out.numel() != n or not out.is_contiguous():
            raise ValueError("bad output tensor")
        return out

    def _call(self, name, x, y):
        fn = getattr(lib(), name)
        _check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())), name)

    # -- transforms ----------------------------------------------------------
    def forward(self, fhat, out=None):
        """f = Lambda fhat (M values, caller's point order)."""
        x = self._in(fhat, self.nc, "fhat")
        y = self._out(self.M, out)
        self._call("sgl_forward", x, y)
        return y

    def adjoint(self, f, out=None):
        """fhat = Lambda^H f (Nc values, coefficient order mu)."""
        x = self._in(f, self.M, "f")
        y = self._out(self.nc, out)
        self._call("sgl_adjoint", x, y)
        return y

    def forward_adjoint(self, fhat, y, out=None, out_adj=None):
        """(Lambda fhat, Lambda^H y), the two computed concurrently on two streams."""
        fh = self._in(fhat, self.nc, "fhat")
        yy = self._in(y, self.M, "y")
        f = self._out(self.M, out)
        g = self._out(self.nc, out_adj)
        _check(lib().sgl_forward_adjoint(self._h, ctypes.c_void_p(fh.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                         ctypes.c_void_p(yy.data_ptr()), ctypes.c_void_p(g.data_ptr())),
               "sgl_forward_adjoint")
        return f, g

    def conv_forward(self, fhat, out=None):
        x = self._in(fhat, self.nc, "fhat")
        n = self.eta_shape[0] * self.eta_shape[1] * self.eta_shape[2]
        y = self._out(n, out)
        self._call("sgl_conv_forward", x, y)
        return y.view(self.eta_shape)

    def conv_adjoint(self, eta, out=None):
        n = self.eta_shape[0] * self.eta_shape[1] * self.eta_shape[2]
        x = self._in(eta.reshape(-1), n, "eta")
        y = self._out(self.nc, out)
        self._call("sgl_conv_adjoint", x, y)
        return y

    def nfft_forward(self, eta, out=None):
        n = self.eta_shape[0] * self.eta_shape[1] * self.eta_shape[2]
        x = self._in(eta.reshape(-1), n, "eta")
        y = self._out(self.M, out)
        self._call("sgl_nfft_forward", x, y)
        return y

    def nfft_adjoint(self, f, out=None):
        n = self.eta_shape[0] * self.eta_shape[1] * self.eta_shape[2]
        x = self._in(f, self.M, "f")
        y = self._out(n, out)
        self._call("sgl_nfft_adjoint", x, y)
        return y.view(self.eta_shape)

    def grad_points(self, fhat, points, g, out=None):
        """Re(conj(g_i) d f_i / d x_i), (M, 3): the gradient with respect to the
        point positions (rho fixed) of a real loss with dL/d conj(f) = g; points
        are the tensor the plan was made with."""
        x = self._in(fhat, self.nc, "fhat")
        gg = self._in(g, self.M, "g")
        if not points.is_cuda or points.dtype != self.real_dtype or points.shape != (self.M, 3):
            raise ValueError(f"points must be the plan's CUDA tensor (M, 3) of {self.real_dtype}")
        points = points.contiguous()
        if out is None:
            out = self._torch.empty((self.M, 3), dtype=self.real_dtype, device=self.device)
        elif out.dtype != self.real_dtype or out.shape != (self.M, 3) or not out.is_contiguous():
            raise ValueError("bad output tensor")
        _check(lib().sgl_grad_points(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(points.data_ptr()),
                                     ctypes.c_void_p(gg.data_ptr()), ctypes.c_void_p(out.data_ptr())),
               "sgl_grad_points")
        return out

    def cgnr(self, y, weights=None, x0=None, maxiter=100, tol=1e-6):
        """Weighted CGNR for min sum_i w_i |y_i - (Lambda fhat)_i|^2 (the
        inverse transform).  Returns (fhat, info) with info = {iterations,
        rel_normal_residual, weighted_residual_norm}; x0 defaults to zero."""
        yy = self._in(y, self.M, "y")
        w = None
        if weights is not None:
            if not weights.is_cuda or weights.dtype != self.real_dtype or weights.numel() != self.M:
                raise ValueError(f"weights must be a CUDA {self.real_dtype} tensor with {self.M} elements")
            w = weights.contiguous()
        x = self._torch.zeros(self.nc, dtype=self.complex_dtype, device=self.device)
        if x0 is not None:
            x.copy_(self._in(x0, self.nc, "x0"))
        info = (ctypes.c_double * 3)()
        _check(lib().sgl_cgnr(self._h, ctypes.c_void_p(yy.data_ptr()),
                              ctypes.c_void_p(w.data_ptr()) if w is not None else None,
                              ctypes.c_void_p(x.data_ptr()), int(maxiter), float(tol), info), "sgl_cgnr")
        return x, {"iterations": int(info[0]), "rel_normal_residual": info[1], "weighted_residual_norm": info[2]}

    def cgne(self, y, x0=None, maxiter=100, tol=1e-6):
        """CGNE for the minimum-norm solution of Lambda fhat = y (fewer samples
        than coefficients).  Returns (fhat, info) with info = {iterations,
        rel_residual, norm}; x0 defaults to zero."""
        yy = self._in(y, self.M, "y")
        x = self._torch.zeros(self.nc, dtype=self.complex_dtype, device=self.device)
        if x0 is not None:
            x.copy_(self._in(x0, self.nc, "x0"))
        info = (ctypes.c_double * 3)()
        _check(lib().sgl_cgne(self._h, ctypes.c_void_p(yy.data_ptr()), ctypes.c_void_p(x.data_ptr()), int(maxiter),
                              float(tol), info), "sgl_cgne")
        return x, {"iterations": int(info[0]), "rel_residual": info[1], "norm": info[2]}

    def close(self):
        if getattr(self, "_h", None):
            lib().sgl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@functools.lru_cache(maxsize=None)
def _autograd():
    import torch

    class SGLTransform(torch.autograd.Function):
        """f = Lambda(x) fhat for the points of `plan`, differentiable in fhat
        (backward: sgl_adjoint) and in the point positions (backward:
        sgl_grad_points, with the plan's rho held fixed).  The plan fixes the
        points: after moving them, make a new plan."""

        @staticmethod
        def forward(ctx, fhat, points, plan):
            ctx.plan = plan
            ctx.save_for_backward(fhat, points)
            return plan.forward(fhat.detach())

        @staticmethod
        def backward(ctx, g):
            fhat, points = ctx.saved_tensors
            plan = ctx.plan
            g = g.contiguous().to(plan.complex_dtype)
            gf = plan.adjoint(g) if ctx.needs_input_grad[0] else None
            gx = plan.grad_points(fhat.detach(), points.detach(), g) if ctx.needs_input_grad[1] else None
            return gf, gx, None

    return SGLTransform


def transform(fhat, points, plan):
    """Differentiable f = Lambda(points) fhat through `plan` (torch.autograd)."""
    return _autograd().apply(fhat, points, plan)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class WeightNet:
    """Learned density-compensation weights for ``Plan.cgnr`` (include/sgl.h):
    w_i = exp(c_i - d_i - |x_i|^2) / M with d_i a histogram log density and
    c = MLP(features), a 4 -> 64 -> 64 -> 1 tanh network in float32.  The last
    layer starts at zero, so an untrained network gives the histogram weights.
    Training (``train``) runs ``sgl_mlp_train_step``: the loss is
    |Lambda^H W Lambda fhat - fhat|^2 / |fhat|^2 over random coefficient vectors.
    """

    def __init__(self, device=None, seed=0):
        import torch

        self._torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        n = int(lib().sgl_mlp_num_params())
        g = torch.Generator().manual_seed(int(seed))
        H, F = 64, 4
        w1 = (torch.rand(H * F, generator=g) * 2 - 1) / F ** 0.5
        b1 = (torch.rand(H, generator=g) * 2 - 1) / F ** 0.5
        w2 = (torch.rand(H * H, generator=g) * 2 - 1) / H ** 0.5
        b2 = (torch.rand(H, generator=g) * 2 - 1) / H ** 0.5
        p = torch.cat([w1, b1, w2, b2, torch.zeros(H + 1)])
        assert p.numel() == n
        self.params = p.to(self.device, torch.float32)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def features(self, plan, points):
        """(M, 4) float32 features of the plan's points (the tensor the plan was made from)."""
        if points.dtype != plan.real_dtype or points.shape != (plan.M, 3) or not points.is_cuda:
            raise ValueError("points must be the plan's (M, 3) CUDA tensor")
        pts = points.contiguous()
        feat = self._torch.empty((plan.M, 4), dtype=self._torch.float32, device=plan.device)
        _check(lib().sgl_point_features(plan._h, _ptr(pts), _ptr(feat)), "sgl_point_features")
        return feat

    def c(self, plan, feat):
        out = self._torch.empty(plan.M, dtype=self._torch.float32, device=plan.device)
        _check(lib().sgl_mlp_forward(plan._h, _ptr(self.params), _ptr(feat), _ptr(out)), "sgl_mlp_forward")
        return out

    def weights(self, plan, feat, learned=True):
        """Weights in the plan's real dtype; learned=False gives the histogram weights (c = 0)."""
        c = self.c(plan, feat) if learned else None
        w = self._torch.empty(plan.M, dtype=plan.real_dtype, device=plan.device)
        _check(lib().sgl_mlp_weights(plan._h, _ptr(c), _ptr(feat), _ptr(w)), "sgl_mlp_weights")
        return w

    def train_step(self, plan, feat, fhats, lr=1e-3):
        """One Adam step on the coefficient vectors fhats (nbatch x num_coeffs); returns the loss."""
        if fhats.dtype != plan.complex_dtype or fhats.numel() % plan.nc or not fhats.is_cuda:
            raise ValueError("fhats must be CUDA (nbatch, num_coeffs) of the plan's complex dtype")
        fhats = fhats.contiguous()
        self.step += 1
        loss = ctypes.c_double()
        _check(lib().sgl_mlp_train_step(plan._h, _ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(feat),
                                        _ptr(fhats), fhats.numel() // plan.nc, float(lr), self.step,
                                        ctypes.byref(loss)), "sgl_mlp_train_step")
        return loss.value

    def train(self, plan, feat, steps=100, nbatch=4, lr=1e-3, decay=1.5, seed=0):
        """Train on random coefficient vectors, Re and Im iid N(0, 1) times n^-decay
        (n the first index of the coefficient); returns the losses."""
        torch = self._torch
        g = torch.Generator(device=plan.device).manual_seed(int(seed))
        n = torch.arange(1, plan.B + 1, device=plan.device)
        scale = torch.repeat_interleave(n, n * n).to(plan.real_dtype) ** (-float(decay))
        losses = []
        for _ in range(int(steps)):
            re = torch.randn((nbatch, plan.nc), generator=g, device=plan.device, dtype=plan.real_dtype)
            im = torch.randn((nbatch, plan.nc), generator=g, device=plan.device, dtype=plan.real_dtype)
            losses.append(self.train_step(plan, feat, torch.complex(re * scale, im * scale), lr))
        return losses


class Batch:
    """The forward and/or adjoint of several plans recorded once as one HIP graph
    (include/sgl.h, sgl_batch_create) and replayed by ``run()`` with one launch.

    plans: list of Plan; fhats / outs: per-plan coefficient inputs and point
    outputs of the forward (or None); ys / ghats: point inputs and coefficient
    outputs of the adjoint (or None).  The tensors are held for the batch's life:
    every run reads and writes those same buffers.
    """

    def __init__(self, plans, fhats=None, outs=None, ys=None, ghats=None, nstreams=4, stream=None):
        import torch

        n = len(plans)
        self.plans = list(plans)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._keep = []

        def arr(ts, what, counts):
            if ts is None:
                return None
            if len(ts) != n:
                raise ValueError(f"{what}: one tensor per plan")
            for t, p, c in zip(ts, plans, counts):
                if not t.is_cuda or t.dtype != p.complex_dtype or t.numel() != c(p) or not t.is_contiguous():
                    raise ValueError(f"{what}: contiguous CUDA {p.complex_dtype} tensors of the plan's size")
            self._keep.extend(ts)
            return (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])

        nc, m = (lambda p: p.nc), (lambda p: p.M)
        a_fh, a_f = arr(fhats, "fhats", [nc] * n), arr(outs, "outs", [m] * n)
        a_y, a_g = arr(ys, "ys", [m] * n), arr(ghats, "ghats", [nc] * n)
        hs = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
        h = ctypes.c_void_p()
        _check(lib().sgl_batch_create(ctypes.byref(h), hs, n, a_fh, a_f, a_y, a_g, int(nstreams),
                                      ctypes.c_void_p(self.stream.cuda_stream)), "sgl_batch_create")
        self._h = h

    def run(self):
        _check(lib().sgl_batch_run(self._h), "sgl_batch_run")

    def close(self):
        if getattr(self, "_h", None):
            lib().sgl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
