"""Throughput of the fast SGL Fourier transform for scattered data on one MI355X.

One step = one forward (f = Lambda fhat) then one adjoint (fhat = Lambda^H y)
over the whole workload on the plan's stream, inputs resident in HBM.
Default workload: B=64, M=4e6 points iid N(0, I/2), coefficients with n^-1.5
decay, FP64 arithmetic throughout (the paper's precision), sigma=2, q=6.
Prints one JSON line with points/s, the roofline position of the dominant
kernel (HIP-event time on the plan's stream), the accuracy against the
direct-sum oracle on a sampled subset, the oracle's own CPU rate, and beside
them the same workload in the FP32 form (matrix-core gather and spread).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scattered points/s fwd+adj at B=64, M=4e6, rel err≤1e-5; frac of HBM roofline"

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_F16_TFLOPS = 2500.0  # dense FP16 matrix cores
MFMA_PEAK_F64_TFLOPS = 78.6    # dense FP64 matrix cores
# FP32 vector FMA issue rate without packed math: 256 CU x 4 SIMD x 16 lanes x
# 2 flop x 2.4 GHz (the build disables packed FP32 instructions).
ALU_PEAK_F32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
ALU_PEAK_F64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="b64_m4e6_f64")
    ap.add_argument("--beside", nargs="*", default=["b64_m4e6_f32", "b64_m4e6_f64_q14"],
                    help="further workloads measured in the same run and reported beside the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--grad", action="store_true",
                    help="time the differentiation step (forward, adjoint and point gradient) instead")
    ap.add_argument("--inverse", action="store_true",
                    help="time the inverse transform (CGNR, plain / histogram / learned weights) instead")
    ap.add_argument("--batch", action="store_true",
                    help="time 64 heterogeneous transforms (forward + adjoint) eagerly and as one HIP graph")
    ap.add_argument("--conv-split16", action="store_true",
                    help="conversion products on the FP16 matrix cores with hi/lo split operands")
    ap.add_argument("--sequential", action="store_true",
                    help="only the headline workload, without the concurrent paired call (profiled runs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--check-points", type=int, default=2000)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied by a plain device copy before the timed region (counter calibration)")
    ap.add_argument("--summarize", nargs=3, metavar=("KT_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="summarize rocprofv3 output directories into --summary-out and exit")
    ap.add_argument("--summary-out", default=None,
                    help="summary file (default profiles/nfsglft_<workload>.md)")
    return ap.parse_args()


PROFILE_COMMAND = ("rocprofv3 {mode} -T -f csv -d gpurun_out/prof_{name}_{tag} -o {tag} -- python3 bench.py "
                   "--workload {name} --steps {steps} --warmup 1 --no-cpu-baseline --check-points 0 "
                   "--copy-calibration 256 --sequential")


def profile_command(workload, **kw):
    """The rocprofv3 command line of one profiled run of this script."""
    return PROFILE_COMMAND.format(name=workload, **kw)


def spread_flops(q):
    """Algorithmic flops per point of the windowed gather (or scatter): the
    (2q)^3 window taps, each a complex-by-real multiply-add (4 flop)."""
    return 4 * (2 * q) ** 3


def fft_bytes(info, B, cb):
    """Algorithmic HBM bytes of the 3D FFT passes: each pass reads its nonzero
    input rows once and writes its needed output rows once.  The passes run
    along dimensions 1, 0, 2 (forward) and 2, 0, 1 (adjoint); eta and the
    intermediates are FP64, the grid (forward output, folded adjoint input) is
    in the plan's precision."""
    n0, n1, n2 = 4 * B, 2 * B, 2 * B
    N2, E0, E1 = info["N2"], info["E0"], info["E1"]
    eta, t1, t2, grid = n0 * n1 * n2, n0 * E1 * n2, E0 * E1 * n2, E0 * E1 * N2
    return {"fft_A": 16 * (eta + t1), "fft_B": 16 * (t1 + t2), "fft_C": 16 * t2 + cb * grid,
            "fft_Ch": cb * grid + 16 * t2, "fft_Bh": 16 * (t2 + t1), "fft_Ah": 16 * (t1 + eta)}


def cpu_baseline(B, pts, fh, y, seconds):
    """The oracle as it stands (direct O(B^3) sum per point, OpenMP), forward +
    adjoint on a bounded sample of the same workload."""
    import oracle

    threads = oracle.max_threads()
    m0 = 500
    t = time.perf_counter()
    oracle.direct_forward(B, pts[:m0], fh)
    oracle.direct_adjoint(B, pts[:m0], y[:m0])
    dt = time.perf_counter() - t
    m = m0
    # the probe's rate is low (thread start-up): size up again from each run, at most twice
    for _ in range(2):
        if dt >= seconds / 2 or m >= len(pts):
            break
        m = int(min(len(pts), max(m0, m * seconds / max(dt, 1e-6))))
        t = time.perf_counter()
        oracle.direct_forward(B, pts[:m], fh)
        oracle.direct_adjoint(B, pts[:m], y[:m])
        dt = time.perf_counter() - t
    return {"value": m / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"first {m} of the {len(pts)} workload points, forward + adjoint, {dt:.1f} s"}


def accuracy(B, plan, pts_used, fh_used, f_gpu, y, prec, m, torch, cdt):
    """Relative l2/linf error against the direct sum on m sampled points
    (forward) and for the adjoint of samples supported on those points."""
    import oracle

    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(len(pts_used), m, replace=False))
    f0 = oracle.direct_forward(B, pts_used[idx], fh_used)
    fs = f_gpu[idx]
    ys = np.zeros(len(pts_used), dtype=np.complex128)
    ys[idx] = y[idx]
    if prec == "f32":
        ys = ys.astype(np.complex64).astype(np.complex128)
    g = plan.adjoint(torch.from_numpy(ys).to("cuda", cdt))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    g0 = oracle.direct_adjoint(B, pts_used[idx], ys[idx])
    n2 = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    ni = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    return {"fwd_rel_l2": n2(fs, f0), "fwd_rel_linf": ni(fs, f0), "adj_rel_l2": n2(g, g0),
            "adj_rel_linf": ni(g, g0), "sample_points": m}


# ---------------------------------------------------------------- profiles

STAGE_KERNEL_VALU = {"gather": "k_gather_tiled", "scatter": "k_spread_rows", "fold": "k_fold_staging"}
STAGE_KERNEL_DIRECT = {"gather": "k_gather_slab", "scatter": "k_scatter_owned", "fold": "k_fold_owned"}
STAGE_KERNEL_MFMA = {"gather": "k_gather_mfma", "scatter": "k_spread_mfma", "fold": "k_fold_tiles8"}
STAGE_KERNEL_MFMA64 = {"gather": "k_gather_tiled", "scatter": "k_spread_mfma64", "fold": "k_fold_tiles8"}
KERNEL_SOURCE = {"k_gather_tiled": "sgl_spread.hip", "k_spread_rows": "sgl_spread.hip",
                 "k_fold_staging": "sgl_spread.hip", "k_gather_mfma": "sgl_spread.hip",
                 "k_spread_mfma": "sgl_spread.hip", "k_fold_tiles8": "sgl_spread.hip", "k_fft": "sgl_fft.hip"}


def stage_kernels(info):
    """Kernel that runs each gather/scatter/fold stage of a plan (plan info)."""
    k = dict({1: STAGE_KERNEL_DIRECT, 2: STAGE_KERNEL_MFMA, 3: STAGE_KERNEL_MFMA64}.get(info["gather_mode"],
                                                                                     STAGE_KERNEL_VALU))
    if (info["L0"], info["L1"], info["L2"]) != (8, 8, 8):
        k["fold"] = "k_fold_staging"
    return k


def source_digest(kernel):
    """Digest of the kernel's source file with comments and whitespace removed,
    so that a profile stays valid across edits of comments only."""
    import hashlib
    import re

    path = os.path.join(ROOT, "paper_1809_10786_amd", "csrc", KERNEL_SOURCE.get(kernel, "sgl_spread.hip"))
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256("".join(text.split()).encode()).hexdigest()[:16]


def summarize_profiles(kt_dir, fetch_dir, write_dir, out_md, workload):
    """Write a markdown summary of one rocprofv3 kernel-trace/stats run and two
    counter runs (FETCH_SIZE, WRITE_SIZE) of this script.  The counters are
    scaled by what they read for the plain 256 MiB device copy that the
    profiled command performs (--copy-calibration 256)."""
    import csv
    import glob

    def one(pattern):
        d, name = os.path.split(pattern)
        hits = sorted(glob.glob(os.path.join(d, "**", name), recursive=True))
        if not hits:
            raise FileNotFoundError(pattern)
        return hits[0]

    stats = list(csv.DictReader(open(one(os.path.join(kt_dir, "*_kernel_stats.csv")))))
    counters = {}
    for d, name in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        rows = list(csv.DictReader(open(one(os.path.join(d, "*_counter_collection.csv")))))
        calib = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        calib = max(calib) if calib else 0.0
        factor = (256 * 1024) / calib if calib else 1.0
        per = {}
        for r in rows:
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * factor * 1024)
        counters[name] = (factor, {k: sum(v) / len(v) for k, v in per.items()})
    lines = [f"# rocprofv3 summary: {os.path.basename(out_md)[:-3]}", "",
             "Command (kernel trace and statistics):", "", "```",
             profile_command(workload, mode="--kernel-trace --stats", tag="kt", steps=5),
             "```", "", "Counter runs (one counter each):", "", "```",
             profile_command(workload, mode="--pmc FETCH_SIZE", tag="fetch", steps=2),
             profile_command(workload, mode="--pmc WRITE_SIZE", tag="write", steps=2),
             "```", "",
             f"Counter calibration on the plain 256 MiB copy: FETCH_SIZE x {counters['FETCH_SIZE'][0]:.3f}, "
             f"WRITE_SIZE x {counters['WRITE_SIZE'][0]:.3f} (scaled bytes below).", "",
             "| kernel | calls | avg us | share % | HBM read MB/launch | HBM write MB/launch | GB/s |",
             "|---|---|---|---|---|---|---|"]
    for r in stats:
        k = r["Name"]
        avg_us = float(r["AverageNs"]) / 1e3
        rd = counters["FETCH_SIZE"][1].get(k)
        wr = counters["WRITE_SIZE"][1].get(k)
        gbs = ((rd or 0) + (wr or 0)) / (avg_us * 1e-6) / 1e9 if rd is not None else None
        lines.append(f"| {k} | {r['Calls']} | {avg_us:.1f} | {float(r['Percentage']):.2f} | "
                     f"{'' if rd is None else f'{rd / 1e6:.1f}'} | {'' if wr is None else f'{wr / 1e6:.1f}'} | "
                     f"{'' if gbs is None else f'{gbs:.0f}'} |")
    lines += ["", "Machine-readable (bytes per launch, with the digest of the kernel's source file):", ""]
    for k in sorted(set(STAGE_KERNEL_MFMA.values()) | set(STAGE_KERNEL_VALU.values()) |
                    set(STAGE_KERNEL_MFMA64.values()) | set(STAGE_KERNEL_DIRECT.values())):
        rd = counters["FETCH_SIZE"][1].get(k)
        wr = counters["WRITE_SIZE"][1].get(k)
        if rd is not None and wr is not None:
            lines.append(f"    traffic {k} read={rd:.0f} write={wr:.0f} source={source_digest(k)}")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profiled_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed profile summary, or
    None if there is none or the kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"nfsglft_{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) == 5 and parts[0] == "traffic" and parts[1] == kernel:
            kv = dict(p.split("=") for p in parts[2:])
            if kv["source"] != source_digest(kernel):
                return None
            return float(kv["read"]) + float(kv["write"])
    return None


def bench_grad(a, torch, wl, sgl):
    """Differentiation step of f = Lambda(x) fhat: forward, adjoint (dL/dfhat)
    and point gradient (dL/dx, rho fixed) per step, with the point gradient of
    sampled points against the oracle's analytic gradient."""
    from oracle import stepwise as sw

    w, pts, fh, y = wl.workload(a.workload, seed=0)
    B, M, q, prec = w["B"], w["M"], w["q"], w["prec"]
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    pu = pts.astype(np.float32).astype(np.float64) if prec == "f32" else pts
    rho = 1.0001 * float(np.linalg.norm(pu, axis=1).max())
    P = torch.from_numpy(pu).to("cuda", rdt)
    dfh = torch.from_numpy(fh).to("cuda", cdt)
    dy = torch.from_numpy(y).to("cuda", cdt)
    plan = sgl.Plan(P, B, sigma=w["sigma"], q=q, rho=rho, precision=prec)
    f = torch.empty(M, dtype=cdt, device="cuda")
    gf = torch.empty(plan.nc, dtype=cdt, device="cuda")
    gx = torch.empty((M, 3), dtype=rdt, device="cuda")
    for _ in range(a.warmup):
        plan.forward(dfh, out=f)
        plan.adjoint(dy, out=gf)
        plan.grad_points(dfh, P, dy, out=gx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        plan.forward(dfh, out=f)
        plan.adjoint(dy, out=gf)
        plan.grad_points(dfh, P, dy, out=gx)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.steps
    print(f"[bench] grad {a.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    idx = np.sort(np.random.default_rng(5).choice(M, 40, replace=False))
    fhu = fh.astype(np.complex64).astype(np.complex128) if prec == "f32" else fh
    yu = y.astype(np.complex64).astype(np.complex128) if prec == "f32" else y
    g0 = np.real(np.conj(yu[idx])[:, None] * sw.forward_grad(B, pu[idx], fhu))
    gg = gx.cpu().numpy().astype(np.float64)[idx]
    gerr = float(np.abs(gg - g0).max() / np.abs(g0).max())
    print(json.dumps({
        "metric": "points/s of the differentiation step (f, dL/dfhat, dL/dx)",
        "value": M / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "dtype": prec, "data": "synthetic",
        "config": {"workload": a.workload, "B": B, "M": M, "q": q, "rho": rho},
        "grad_points_rel_err_max": gerr, "sample_points": len(idx)}), flush=True)


def bench_inverse(a, torch, wl, sgl):
    """Inverse transform, CGNR with W = I (plain), histogram density weights and
    learned weights (network trained with the native step on other clouds of
    the same distribution), 1 % noise:
    * the clustered cloud (B=32, M=3e5, eight Gaussian clusters): the clusters
      leave part of the weighted support unsampled, so the comparison stops at
      a normal residual of 1e-3;
    * a cloud covering the ball of radius 5 (B=12, M=2e4, density falling as
      1/r): iterations and time to a normal residual of 1e-6;
    and CGNE (the minimum-norm solution, Section 2) for fewer samples than
    coefficients (B=8, 100 Gaussian points) to a residual of 1e-6."""
    cases = (("b32_m3e5_clustered_f64", 1e-3, [1], 150, 2, 1e-2),
             ("b12_m2e4_centered5_f64", 1e-6, [320, 321], 300, 4, 5e-3))
    out = {}
    for name, tol, train_seeds, steps, nbatch, lr in cases:
        w, pts, fh, _ = wl.workload(name, seed=0)
        B, M, q, prec = w["B"], w["M"], w["q"], w["prec"]
        rdt = torch.float64 if prec == "f64" else torch.float32
        cdt = torch.complex128 if prec == "f64" else torch.complex64
        net = sgl.WeightNet(seed=4)
        plans_t, feats_t = [], []
        for s_ in train_seeds:
            Pt = torch.from_numpy(wl.make_points(w["points"], M, s_)).to("cuda", rdt)
            plans_t.append(sgl.Plan(Pt, B, sigma=w["sigma"], q=q, precision=prec))
            feats_t.append(net.features(plans_t[-1], Pt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = []
        per = steps // (len(plans_t) * 3)
        for r in range(len(plans_t) * 3):
            k = r % len(plans_t)
            losses += net.train(plans_t[k], feats_t[k], steps=per, nbatch=nbatch, lr=lr, decay=w["decay"], seed=5 + r)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        for pt in plans_t:
            pt.close()
        print(f"[bench] inverse {name}: trained {len(losses)} steps in {train_s:.2f} s, loss {losses[0]:.4g} -> "
              f"{losses[-1]:.4g}", file=sys.stderr, flush=True)
        P = torch.from_numpy(pts).to("cuda", rdt)
        plan = sgl.Plan(P, B, sigma=w["sigma"], q=q, precision=prec)
        F = net.features(plan, P)
        fstar = torch.from_numpy(fh).to("cuda", cdt)
        y0 = plan.forward(fstar)
        rms = torch.sqrt(torch.mean(torch.abs(y0) ** 2))
        g = torch.Generator(device="cuda").manual_seed(7)
        noisy = y0 + torch.complex(torch.randn(M, generator=g, device="cuda", dtype=rdt),
                                   torch.randn(M, generator=g, device="cuda", dtype=rdt)) * (0.01 * rms / 2 ** 0.5)
        res = {"B": B, "M": M, "q": q, "tol": tol, "train_steps": len(losses), "train_seconds": train_s}
        for data, y in (("noisy", noisy), ("exact", y0)):
            for label, wt in (("plain", None), ("histogram", net.weights(plan, F, learned=False)),
                              ("learned", net.weights(plan, F))):
                plan.cgnr(y, weights=wt, maxiter=5, tol=tol)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = plan.cgnr(y, weights=wt, maxiter=20000, tol=tol)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                err = float(torch.linalg.vector_norm(x - fstar) / torch.linalg.vector_norm(fstar))
                key = label if data == "noisy" else f"{label}_exact_samples"
                res[key] = {"iterations": info["iterations"], "seconds": dt,
                            "ms_per_iteration": dt * 1e3 / max(info["iterations"], 1), "rel_error_vs_truth": err,
                            "rel_normal_residual": info["rel_normal_residual"]}
                print(f"[bench] inverse {name} {key}: {res[key]}", file=sys.stderr, flush=True)
        plan.close()
        out[name] = res
    # CGNE: fewer samples than coefficients (the under-determined systems of
    # scattered SGL samples are ill-conditioned: cond(Lambda) is about 4e3 at
    # B = 8 on 100 Gaussian points and above 1e7 at B = 12 on 400)
    B, M = 8, 100
    P = torch.from_numpy(wl.gaussian_points(M, 160)).to("cuda", torch.float64)
    plan = sgl.Plan(P, B, q=12)
    fstar = torch.from_numpy(wl.coefficients(B, 161)).to("cuda", torch.complex128)
    y = plan.forward(fstar)
    plan.cgne(y, maxiter=5, tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = plan.cgne(y, maxiter=20000, tol=1e-6)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["cgne_b8_m100_gaussian_f64"] = {"B": B, "M": M, "iterations": info["iterations"], "seconds": dt,
                                        "rel_residual": info["rel_residual"]}
    print(f"[bench] cgne {out['cgne_b8_m100_gaussian_f64']}", file=sys.stderr, flush=True)
    plan.close()
    cov = out["b12_m2e4_centered5_f64"]
    print(json.dumps({
        "metric": "CGNR seconds to normal residual 1e-6 with learned weights (covering cloud)",
        "value": cov["learned"]["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "b12_m2e4_centered5_f64", "noise": 0.01},
        "solves": out}), flush=True)


def bench_batch(a, torch, wl, sgl):
    """64 transforms, B uniform in [16, 64] (FFT lengths padded where sigma n has
    a prime factor above 5), M log-uniform in [1e5, 2e6], mixed points, FP32,
    coefficients with n^-1 decay:
    forward + adjoint of all of them per step, eagerly (one plan after another
    on one stream) and replayed as one HIP graph over 4 branches."""
    specs = wl.batch_specs(64, seed=0)
    total = sum(m for _, m in specs)
    plans, fh, ys, outs, ghs = [], [], [], [], []
    t0 = time.perf_counter()
    for k, (B, M) in enumerate(specs):
        P = torch.from_numpy(wl.mixed_points(M, 1000 + k)).to("cuda", torch.float32)
        plans.append(sgl.Plan(P, B, precision="f32"))
        del P
        fh.append(torch.from_numpy(wl.coefficients(B, 2000 + k, decay=1.0)).to("cuda", torch.complex64))
        ys.append(torch.from_numpy(wl.samples(M, 3000 + k)).to("cuda", torch.complex64))
        outs.append(torch.empty(M, dtype=torch.complex64, device="cuda"))
        ghs.append(torch.empty(plans[-1].nc, dtype=torch.complex64, device="cuda"))
    torch.cuda.synchronize()
    print(f"[bench] batch: {len(specs)} plans, {total} points, planned in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    def eager():
        for p, f, o, y, g in zip(plans, fh, outs, ys, ghs):
            p.forward(f, out=o)
            p.adjoint(y, out=g)

    t0 = time.perf_counter()
    b = sgl.Batch(plans, fh, outs, ys, ghs, nstreams=4)
    capture_ms = (time.perf_counter() - t0) * 1e3
    res = {}
    for label, fn in (("eager", eager), ("graph", b.run)):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        res[label] = (time.perf_counter() - t0) * 1e3 / a.steps
        print(f"[bench] batch {label}: {res[label]:.3f} ms/step", file=sys.stderr, flush=True)
    b.close()
    ms = res["graph"]
    print(json.dumps({
        "metric": "scattered points/s fwd+adj over a batch of 64 heterogeneous transforms", "value": total / (ms * 1e-3),
        "unit": "points/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 transforms, B in [16, 64], M log-uniform in [1e5, 2e6], mixed points",
                   "total_points": total, "nstreams": 4, "capture_ms": capture_ms},
        "eager_ms_per_step": res["eager"], "graph_ms_per_step": ms}), flush=True)


def measure(a, torch, wl, sgl, name, check_points, conv_split16=False, paired=True):
    """Plan the workload, time K steps (forward then adjoint on the plan's
    stream; also the concurrent paired call), time every stage with HIP events
    on a second pass, and check sampled outputs against the oracle."""
    w, pts, fh, y = wl.workload(name, seed=0)
    B, M, q, prec = w["B"], w["M"], w["q"], w["prec"]
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    cb = 16 if prec == "f64" else 8
    print(f"[bench] workload {name}: B={B} M={M} q={q} {prec}", file=sys.stderr, flush=True)

    dpts = torch.from_numpy(pts).to("cuda", rdt)
    dfh = torch.from_numpy(fh).to("cuda", cdt)
    dy = torch.from_numpy(y).to("cuda", cdt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = sgl.Plan(dpts, B, sigma=w["sigma"], q=q, precision=prec, conv_split16=conv_split16)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    del dpts
    info = plan.info()
    print(f"[bench] plan {plan_ms:.1f} ms, rho={plan.rho:.4f}, info={info}", file=sys.stderr, flush=True)

    if a.copy_calibration > 0:
        # a plain copy kernel of known size: reads and writes copy_calibration MiB each
        src = torch.ones(a.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] copy calibration: 3 x {a.copy_calibration} MiB", file=sys.stderr, flush=True)

    f = torch.empty(M, dtype=cdt, device="cuda")
    g = torch.empty(plan.nc, dtype=cdt, device="cuda")
    for _ in range(a.warmup):
        plan.forward(dfh, out=f)
        plan.adjoint(dy, out=g)
        if paired:
            plan.forward_adjoint(dfh, dy, out=f, out_adj=g)  # the first call sets up the second stream
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    def timed(fn):
        """Mean ms per step over exactly K steps (host clock, synchronised on
        both sides) and the median of the per-step HIP-event times (events at
        the step boundaries on the plan's stream)."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for k in range(a.steps):
            fn()
            ev[k + 1].record()
        torch.cuda.synchronize()
        mean = (time.perf_counter() - t0) * 1e3 / a.steps
        per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(a.steps))
        return mean, per[len(per) // 2]

    def sequential():
        plan.forward(dfh, out=f)
        plan.adjoint(dy, out=g)

    # the step: forward then adjoint on the plan's stream (a dependent caller's
    # order, as in CGNR), no stage timers
    ms_seq, med_seq = timed(sequential)
    ms_pair = med_pair = None
    if paired:
        # the same two transforms on independent inputs, run concurrently on two streams
        ms_pair, med_pair = timed(lambda: plan.forward_adjoint(dfh, dy, out=f, out_adj=g))
    # per-kernel durations: HIP events on the plan's stream over a second pass
    # of the same K steps, one stage at a time
    plan.profile(True)
    plan.stage_times(reset=True)
    timed(sequential)
    stages = plan.stage_times(reset=True)
    plan.profile(False)
    print(f"[bench] {name} {a.steps} steps: forward then adjoint {ms_seq:.3f} ms/step (median {med_seq:.3f}), "
          f"{M / (ms_seq * 1e-3):.4g} points/s" +
          (f"; concurrent pair {ms_pair:.3f} ms/step" if paired else ""), file=sys.stderr, flush=True)

    avg = {k: v[0] / v[1] for k, v in stages.items()}
    print(f"[bench] stages (ms/launch): " + ", ".join(f"{k}={v:.4f}" for k, v in avg.items()), file=sys.stderr,
          flush=True)
    dom = max(avg, key=avg.get)
    fb = fft_bytes(info, B, cb)
    kern = stage_kernels(info)
    if dom in ("gather", "scatter"):
        # algorithmic flops per launch: 4 (2q)^3 per point (complex-by-real
        # multiply-adds of the window taps) times the M points of one launch
        flops = spread_flops(q) * M
        achieved = flops / (avg[dom] * 1e-3) / 1e12
        if info["gather_mode"] == 2:
            # the contraction runs on the FP16 matrix cores (hi/lo split operands)
            bound, peak = "mfma", MFMA_PEAK_F16_TFLOPS
        elif info["gather_mode"] == 3:
            # FP64 matrix cores (published dense FP64 peak)
            bound, peak = "mfma", MFMA_PEAK_F64_TFLOPS
        else:
            bound, peak = "alu", ALU_PEAK_F32_TFLOPS if prec == "f32" else ALU_PEAK_F64_TFLOPS
        roof = {"kernel": kern[dom], "bound": bound, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "flop_per_point": spread_flops(q),
                "launch_ms": avg[dom], "traffic": profiled_traffic(name, kern[dom])}
        if prec == "f32":
            roof["frac_of_fp32_vector_peak"] = achieved / ALU_PEAK_F32_TFLOPS
    else:
        byts = fb.get(dom, 0)
        achieved = byts / (avg[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "launch_ms": avg[dom], "traffic": None}
    # HBM fraction of the whole step at algorithmic bytes
    step_bytes = sum(fb.values()) + 2 * M * (cb + 16 + 4)
    acc = None
    if check_points > 0:
        f_host = f.cpu().numpy().astype(np.complex128)
        pts_used = pts.astype(np.float32).astype(np.float64) if prec == "f32" else pts
        fh_used = fh.astype(np.complex64).astype(np.complex128) if prec == "f32" else fh
        acc = accuracy(B, plan, pts_used, fh_used, f_host, y, prec, check_points, torch, cdt)
        print(f"[bench] accuracy {acc}", file=sys.stderr, flush=True)
    res = {"workload": name, "B": B, "M": M, "sigma": w["sigma"], "q": q, "prec": prec, "points": w["points"],
           "coeff_decay": w["decay"], "rho": plan.rho, "plan_ms": plan_ms, "ms_seq": ms_seq,
           "median_ms_seq": med_seq, "ms_pair": ms_pair, "median_ms_pair": med_pair,
           "stages_ms": {k: round(v, 5) for k, v in avg.items()}, "roofline": roof,
           "hbm_frac_step": step_bytes / (ms_seq * 1e-3) / (HBM_PEAK_GBS * 1e9), "rel_err": acc,
           "inputs": (pts, fh, y)}
    plan.close()
    return res


def main():
    a = parse()
    if a.summarize:
        out = a.summary_out or os.path.join(ROOT, "profiles", f"nfsglft_{a.workload}.md")
        summarize_profiles(*a.summarize, out_md=out, workload=a.workload)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(sharding over points is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    import torch

    from tests import workloads as wl
    import paper_1809_10786_amd as sgl

    if a.grad:
        return bench_grad(a, torch, wl, sgl)
    if a.inverse:
        return bench_inverse(a, torch, wl, sgl)
    if a.batch:
        return bench_batch(a, torch, wl, sgl)
    r = measure(a, torch, wl, sgl, a.workload, a.check_points, conv_split16=a.conv_split16,
                paired=not a.sequential)
    pts, fh, y = r.pop("inputs")
    # the same workload in the other forms, beside the headline
    beside = {}
    for extra in ([] if a.sequential else a.beside):
        if extra == a.workload:
            continue
        e = measure(a, torch, wl, sgl, extra, min(a.check_points, 1000))
        e.pop("inputs")
        e["points_per_s"] = e["M"] / (e["ms_seq"] * 1e-3)
        beside[extra] = e

    cpu = None
    if not a.no_cpu_baseline:
        pts_used = pts.astype(np.float32).astype(np.float64) if r["prec"] == "f32" else pts
        fh_used = fh.astype(np.complex64).astype(np.complex128) if r["prec"] == "f32" else fh
        cpu = cpu_baseline(r["B"], pts_used, fh_used, y.astype(np.complex128), a.cpu_seconds)
        print(f"[bench] cpu baseline {cpu}", file=sys.stderr, flush=True)

    ms = r["ms_seq"]
    out = {
        "metric": METRIC,
        "value": r["M"] / (ms * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["prec"],
        "data": "synthetic",
        "config": {"workload": r["workload"], "B": r["B"], "M": r["M"], "sigma": r["sigma"], "q": r["q"],
                   "points": r["points"], "coeff_decay": r["coeff_decay"], "rho": r["rho"],
                   "conversion": "fp16-split-mfma" if a.conv_split16 else "fp64"},
        "roofline": r["roofline"],
        "hbm_frac_step": r["hbm_frac_step"],
        "cpu_baseline": cpu,
        "rel_err": r["rel_err"],
        "step": "forward then adjoint on the plan's stream",
        "median_ms_per_step": r["median_ms_seq"],
        "ms_per_step_concurrent_pair": r["ms_pair"],
        "stage_timing": "HIP events on the plan's stream over a second pass of the same steps, one stage at a time",
        "stages_ms": r["stages_ms"],
        "plan_ms": r["plan_ms"],
        "beside": beside,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
