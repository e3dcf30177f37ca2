"""Batches: the forward and adjoint of several plans recorded as one HIP graph.

* every replay equals each plan's own sgl_forward / sgl_adjoint bit for bit
  (same kernels, same inputs, no atomics), over three replays with eager work
  and new input values between them, for 1 and 4 branches;
* forward-only and adjoint-only batches;
* the batch's results against the direct-sum oracle on sampled points
  (FP64 2e-6, FP32 1e-5 relative l2, the plans' own tolerances at q = 6);
* rule violations: a repeated plan, a plan with profiling on.
"""
import numpy as np
import pytest

import oracle
from tests import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPECS = [(6, 1, "f64"), (8, 777, "f32"), (12, 5_000, "f64"), (16, 20_000, "f32"), (9, 3_001, "f32"),
         (10, 12_345, "f64")]


def say(*a):
    print(*a, flush=True)


def make(seed):
    import paper_1809_10786_amd as sgl

    plans, pts, fh, ys = [], [], [], []
    for k, (B, M, prec) in enumerate(SPECS):
        rt, ct = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
        p = wl.mixed_points(M, seed + k) if M > 1 else np.array([[0.3, -0.2, 0.5]])
        P = torch.from_numpy(p).to("cuda", rt)
        plans.append(sgl.Plan(P, B, precision=prec))
        pts.append(P.cpu().numpy().astype(np.float64))
        fh.append(torch.from_numpy(wl.coefficients(B, seed + 50 + k)).to("cuda", ct))
        ys.append(torch.from_numpy(wl.samples(M, seed + 80 + k)).to("cuda", ct))
    return plans, pts, fh, ys


def eager(plans, fh, ys):
    return [p.forward(f) for p, f in zip(plans, fh)], [p.adjoint(y) for p, y in zip(plans, ys)]


@pytest.mark.parametrize("nstreams", [1, 4])
def test_batch_replays_equal_eager(nstreams):
    import paper_1809_10786_amd as sgl

    say(f"batch nstreams={nstreams}")
    plans, _, fh, ys = make(400)
    outs = [torch.empty(p.M, dtype=p.complex_dtype, device="cuda") for p in plans]
    ghs = [torch.empty(p.nc, dtype=p.complex_dtype, device="cuda") for p in plans]
    b = sgl.Batch(plans, fh, outs, ys, ghs, nstreams=nstreams)
    other = sgl.Plan(torch.from_numpy(wl.gaussian_points(4_000, 9)).to("cuda", torch.float64), 8)
    ofh = torch.from_numpy(wl.coefficients(8, 10)).to("cuda", torch.complex128)
    for rep in range(3):
        if rep == 2:  # new input values in the same buffers
            for k, (f, y) in enumerate(zip(fh, ys)):
                f.copy_(torch.from_numpy(wl.coefficients(plans[k].B, 700 + k)).to(f.dtype))
                y.copy_(torch.from_numpy(wl.samples(plans[k].M, 800 + k)).to(y.dtype))
        b.run()
        torch.cuda.synchronize()
        got_f = [o.clone() for o in outs]
        got_g = [g.clone() for g in ghs]
        other.forward(ofh)  # eager work between replays
        ef, eg = eager(plans, fh, ys)
        torch.cuda.synchronize()
        for k in range(len(plans)):
            assert torch.equal(got_f[k], ef[k]), (rep, k, "forward")
            assert torch.equal(got_g[k], eg[k]), (rep, k, "adjoint")
        say(f"  replay {rep}: {len(plans)} forward + adjoint equal to eager")
    b.close()
    other.close()


def test_one_direction_batches_and_oracle():
    import paper_1809_10786_amd as sgl

    say("forward-only and adjoint-only batches")
    plans, pts, fh, ys = make(410)
    outs = [torch.empty(p.M, dtype=p.complex_dtype, device="cuda") for p in plans]
    ghs = [torch.empty(p.nc, dtype=p.complex_dtype, device="cuda") for p in plans]
    bf = sgl.Batch(plans, fh, outs, nstreams=3)
    ba = sgl.Batch(plans, ys=ys, ghats=ghs, nstreams=2)
    bf.run()
    ba.run()
    torch.cuda.synchronize()
    ef, eg = eager(plans, fh, ys)
    torch.cuda.synchronize()
    for k in range(len(plans)):
        assert torch.equal(outs[k], ef[k]) and torch.equal(ghs[k], eg[k]), k
    # against the oracle: forward on sampled points; adjoint of samples supported
    # on those points only (written into the buffers the batch reads, then replayed)
    rng = np.random.default_rng(3)
    idxs = []
    for k, p in enumerate(plans):
        idx = np.sort(rng.choice(p.M, min(p.M, 300), replace=False))
        idxs.append(idx)
        yk = np.zeros(p.M, dtype=np.complex128)
        yk[idx] = ys[k].cpu().numpy()[idx]
        ys[k].copy_(torch.from_numpy(yk).to("cuda", p.complex_dtype))
    ba.run()
    torch.cuda.synchronize()
    for k, p in enumerate(plans):
        idx = idxs[k]
        tol = 2e-6 if p.precision == "f64" else 1e-5
        fr = oracle.direct_forward(p.B, pts[k][idx], fh[k].cpu().numpy().astype(np.complex128))
        got = outs[k].cpu().numpy()[idx].astype(np.complex128)
        e = np.linalg.norm(got - fr) / np.linalg.norm(fr)
        ar = oracle.direct_adjoint(p.B, pts[k][idx], ys[k].cpu().numpy()[idx].astype(np.complex128))
        ea = np.linalg.norm(ghs[k].cpu().numpy().astype(np.complex128) - ar) / np.linalg.norm(ar)
        say(f"  plan {k} B={p.B} M={p.M} {p.precision}: forward {e:.3g} adjoint {ea:.3g}")
        assert e < tol and ea < tol
    bf.close()
    ba.close()


def test_batch_rejects_repeated_and_profiled_plans():
    import paper_1809_10786_amd as sgl

    plans, _, fh, ys = make(420)
    outs = [torch.empty(p.M, dtype=p.complex_dtype, device="cuda") for p in plans]
    with pytest.raises(sgl.SglError) as ei:
        sgl.Batch([plans[1], plans[1]], [fh[1], fh[1]], [outs[1], outs[1]])
    assert ei.value.status == sgl.SGL_E_INVAL
    plans[2].profile(True)
    with pytest.raises(sgl.SglError) as ei:
        sgl.Batch(plans[:3], fh[:3], outs[:3])
    assert ei.value.status == sgl.SGL_E_INVAL
    plans[2].profile(False)
    b = sgl.Batch(plans[:3], fh[:3], outs[:3])
    b.run()
    torch.cuda.synchronize()
    b.close()


def test_batch_with_padded_fft_lengths():
    """Bandwidths whose FFT lengths are padded (B = 17, 23, 31, 61) in one
    batch: the replay equals each plan's eager calls bit for bit and matches
    the direct sum on sampled points."""
    import paper_1809_10786_amd as sgl

    specs = [(17, 3_000), (23, 5_000), (31, 2_000), (61, 4_000)]
    plans, pts, fh, ys = [], [], [], []
    for k, (B, M) in enumerate(specs):
        p = wl.mixed_points(M, 700 + k)
        pts.append(p)
        plans.append(sgl.Plan(torch.from_numpy(p).to("cuda", torch.float64), B))
        fh.append(torch.from_numpy(wl.coefficients(B, 720 + k, decay=1.0)).to("cuda", torch.complex128))
        ys.append(torch.from_numpy(wl.samples(M, 740 + k)).to("cuda", torch.complex128))
    outs = [torch.empty(p.M, dtype=torch.complex128, device="cuda") for p in plans]
    ghs = [torch.empty(p.nc, dtype=torch.complex128, device="cuda") for p in plans]
    b = sgl.Batch(plans, fh, outs, ys, ghs, nstreams=4)
    b.run()
    torch.cuda.synchronize()
    ef, ea = eager(plans, fh, ys)
    for k, (B, M) in enumerate(specs):
        assert torch.equal(outs[k], ef[k]) and torch.equal(ghs[k], ea[k]), B
        idx = np.sort(np.random.default_rng(750 + k).choice(M, 300, replace=False))
        f0 = oracle.direct_forward(B, pts[k][idx], fh[k].cpu().numpy())
        e = float(np.linalg.norm(outs[k].cpu().numpy()[idx] - f0) / np.linalg.norm(f0))
        say(f"padded batch B={B} N0={plans[k].info()['N0']}: forward on 300 points {e:.3g}")
        assert e < 2e-6
    b.close()
    for p in plans:
        p.close()
