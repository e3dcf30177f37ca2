"""sgl_forward_adjoint: the forward and the adjoint of one plan running
concurrently on two streams give exactly (bit for bit) what sgl_forward and
sgl_adjoint give, over repeated calls with new inputs, with profiling on (one
stream), on a plan whose stream is not the default one and in exact-NDFT
mode, and with the narrow tiled gather of windows too wide for 8^3 tiles;
overlapping buffers are rejected."""
import numpy as np
import pytest

from tests import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("B,M,prec,own_stream,ndft", [(32, 100_000, "f32", False, False),
                                                       (8, 5_001, "f64", True, False),
                                                       (64, 300_000, "f32", True, False),
                                                       (6, 2_000, "f64", False, True)])
def test_forward_adjoint_equals_separate_calls(B, M, prec, own_stream, ndft):
    import paper_1809_10786_amd as sgl

    say(f"forward_adjoint B={B} M={M} {prec} own_stream={own_stream} exact_ndft={ndft}")
    rt, ct = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    P = torch.from_numpy(wl.mixed_points(M, 500)).to("cuda", rt)
    stream = torch.cuda.Stream() if own_stream else None
    plan = sgl.Plan(P, B, precision=prec, stream=stream, exact_ndft=ndft)
    with torch.cuda.stream(plan.stream):
        for rep in range(3):
            fh = torch.from_numpy(wl.coefficients(B, 510 + rep)).to("cuda", ct)
            y = torch.from_numpy(wl.samples(M, 520 + rep)).to("cuda", ct)
            f2, g2 = plan.forward_adjoint(fh, y)
            f1 = plan.forward(fh)
            g1 = plan.adjoint(y)
            torch.cuda.synchronize()
            assert torch.equal(f1, f2) and torch.equal(g1, g2), rep
        plan.profile(True)
        f3, g3 = plan.forward_adjoint(fh, y)
        torch.cuda.synchronize()
        st = plan.stage_times()
        plan.profile(False)
        assert torch.equal(f1, f3) and torch.equal(g1, g3)
        assert "gather" in st or "ndft" in st
        with pytest.raises(sgl.SglError):
            plan.forward_adjoint(fh, y, out=y)  # f would overwrite y while the adjoint reads it
    plan.close()


@pytest.mark.parametrize("B,M,prec,q", [(32, 60_000, "f32", 8), (24, 40_000, "f64", 7)])
def test_forward_adjoint_narrow_tiled_gather(B, M, prec, q):
    """Windows whose 8^3-tile box exceeds the LDS budget run the tiled vector
    gather on smaller tiles; beside the concurrent scatter it takes 256-thread
    workgroups (sixteen lanes per point, fewer point slots), which must give the
    same bits as the separate forward's wide workgroups."""
    import paper_1809_10786_amd as sgl

    say(f"forward_adjoint narrow gather B={B} M={M} {prec} q={q}")
    rt, ct = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    P = torch.from_numpy(wl.mixed_points(M, 530)).to("cuda", rt)
    plan = sgl.Plan(P, B, q=q, precision=prec)
    info = plan.info()
    assert info["gather_mode"] == 0 and (info["L0"], info["L1"], info["L2"]) != (8, 8, 8), info
    with torch.cuda.stream(plan.stream):
        for rep in range(2):
            fh = torch.from_numpy(wl.coefficients(B, 540 + rep)).to("cuda", ct)
            y = torch.from_numpy(wl.samples(M, 550 + rep)).to("cuda", ct)
            f2, g2 = plan.forward_adjoint(fh, y)
            f1 = plan.forward(fh)
            g1 = plan.adjoint(y)
            torch.cuda.synchronize()
            assert torch.equal(f1, f2) and torch.equal(g1, g2), rep
    plan.close()
