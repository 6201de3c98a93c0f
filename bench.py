#!/usr/bin/env python3
"""ADMM iterations per second for Cartesian dynamic parallel MRI on one MI355X.

Workload (default): Algorithm 2 (analysis prior, temporal TV) on a synthetic
256x256 image series of 32 frames with 8 coils, R = 8 variable-density
phase-encode sampling with 12 centre lines and a fresh pattern per frame,
complex Gaussian noise sigma = 0.005, lambda = 0.01, mu2 = 0.1, mu2/mu1 = 0.5.
One step = one ADMM iteration (TV step + exact x-update).  The timed region is
one cs_admm_solve call of --steps iterations from the algorithm's
initialisation (so it includes the H'y setup and the output write), with every
input already in HBM, in the execution form the library's autotuner picked
beforehand, replaying the loop an untimed solve of the same length recorded;
the plan (FP64 factor of (mu I + H'H)^{-1}) is built before it, as the paper
excludes its SVD time.  --repeats further solves of the same length give the
best and median rates (the paper reports the fastest of 10 runs).

Prints one JSON line on stdout.  Also reports the dominant kernel's roofline
(x-update, HBM bound) from HIP events recorded on its launch stream around
every launch of a second timed solve of the same length (events cannot sit
inside a replayed graph, so that solve runs the single-stream phase form), the
24-slice batched-vs-plain comparison, the unrolled derivative's rate, and the
FP64 CPU oracle timed on the host cores on a bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ADMM iter/s @256²×32×8c, plain vs batched+adjoint; % HBM roofline"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
WORKLOADS = {
    "tv256": dict(name="tv-256x256x32-8c", prior="tv"),
    "dft192": dict(name="dft-192x192x40-12c", prior="dft"),
    "tv64": dict(name="tv-64x64x8-4c", prior="tv"),
    "frame192": dict(name="frame-192x192x40-12c", prior="frame", config="dft192"),
    "paper128tv": dict(name="paper-tv-128x128x22-32c", prior="tv"),
    "paper128dft": dict(name="paper-dft-128x128x22-32c", prior="dft"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Fingerprint of the x-update kernels: iterate.hip up to its TV-step section
    (the x-update kernels, their helpers and launchers)."""
    with open(os.path.join(ROOT, "paper_1203_4587_amd", "csrc", "iterate.hip"), encoding="utf-8") as f:
        text = f.read()
    text = text[:text.index("// ---------------------------------------------------------------- TV step")]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


_EIGEN_MARK = "// ---------------------------------------------------------------- x-update, eigen form"
_WAVE2_MARK = "// ---------------------------------------------------------------- x-update, two blocks per wave"


def _iterate_section(start: str, end: str | None) -> str:
    with open(os.path.join(ROOT, "paper_1203_4587_amd", "csrc", "iterate.hip"), encoding="utf-8") as f:
        text = f.read()
    text = text[text.index(start):]
    return text[:text.index(end)] if end else text


def eigen_source_sha() -> str:
    """Fingerprint of the eigen-form x-update kernels: iterate.hip's eigen-form
    section (up to the two-blocks-per-wave section)."""
    return hashlib.sha256(_iterate_section(_EIGEN_MARK, _WAVE2_MARK).encode()).hexdigest()[:16]


def wave2_source_sha() -> str:
    """Fingerprint of the two-blocks-per-wave x-update: iterate.hip from that
    section to the end (its kernel, launchers and the x-update dispatch)."""
    return hashlib.sha256(_iterate_section(_WAVE2_MARK, None).encode()).hexdigest()[:16]


def measured_traffic(kind: str, workload: str, steps: int, sha_fn=None):
    """HBM bytes per launch of `kind` from the committed rocprofv3 PMC summary
    (profiles/<kind>_<workload>_traffic.json), or None when it is missing or
    was taken on a different kernel source.  The single-launch solve's record
    is per iteration and is scaled by the launch's iteration count."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != (sha_fn or kernel_source_sha)() or rec.get("workload") != workload:
        return None
    if "bytes_per_iteration" in rec:
        return int(rec["bytes_per_iteration"] * steps)
    return rec.get("bytes_per_launch")


def cpu_baseline(problem, cols: int, iters: int) -> dict:
    """The FP64 oracle as it stands, timed on the host on a column sample.
    Columns never interact under a temporal prior, so per-iteration time is
    linear in the column count; it is scaled to the full image."""
    import numpy as np
    import oracle as O
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([p.get("num_threads", 1) for p in info] or [os.cpu_count() or 1])
    except Exception:
        cores = os.cpu_count() or 1
    nt, nv, nh = problem.x_true.shape
    sel = np.linspace(0, nh - 1, cols).round().astype(int)
    y = O.measure(problem)
    t0 = time.perf_counter()
    fac = O.BlockFactor(problem.coil, problem.mask, sel)
    t_plan = time.perf_counter() - t0
    Hy = O.adjoint_columns(y, problem.coil, problem.mask, sel)
    t0 = time.perf_counter()
    if problem.prior == "tv":
        O.admm_analysis(Hy, fac, problem.lam, problem.mu, problem.rho, iters)
    else:
        O.admm_synthesis(Hy, fac, problem.lam, problem.mu, iters)
    t_iter = (time.perf_counter() - t0) / iters
    per_full_iter = t_iter * nh / cols
    return {
        "value": 1.0 / per_full_iter,
        "unit": "iter/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": (f"numpy FP64 oracle, {iters} iterations on {cols} of {nh} columns (all {nt} frames), "
                   f"per-iteration time x {nh}/{cols}; plan excluded (eigendecompositions of the "
                   f"sample: {t_plan:.1f} s)"),
    }


def _median(v):
    import statistics
    return statistics.median(v)


def batched_vs_plain(iters: int, reps: int = 3) -> dict:
    """The 24-slice uneven workload (128x96x16 8-coil R=4 up to 256x256x40
    16-coil R=10, both priors): one cs_batch_solve of `iters` iterations per
    slice against the 24 plain cs_admm_solve calls back to back on the same
    plans, each tuned first (cs_plan_tune).  Slice-iterations per second,
    median of `reps` timed runs after one warm-up each."""
    import torch
    from paper_1203_4587_amd import synthetic as S
    from paper_1203_4587_amd.api import Batch, Slice, to_device

    probs = [S.batch_slice(s) for s in range(24)]
    slices = [Slice(to_device(p.coil), to_device(p.mask, dtype=torch.uint8), p.prior, p.mu, p.rho) for p in probs]
    t0 = time.perf_counter()
    batch = Batch(slices)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    plans = [batch.plan(i) for i in range(24)]
    ys = [plans[i].apply_A(to_device(p.x_true)) + to_device(p.noise) for i, p in enumerate(probs)]
    lams = [p.lam for p in probs]
    for i in range(24):
        plans[i].tune(ys[i], lams[i], iters=5)
    outs = [torch.empty(plans[i].image_shape, dtype=torch.complex64, device="cuda") for i in range(24)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return _median(ts)

    t_batch = timed(lambda: batch.solve(ys, lams, iters, outs=outs))
    t_plain = timed(lambda: [plans[i].solve(ys[i], lams[i], iters, out=outs[i]) for i in range(24)])
    alg = 0
    for p in probs:
        nt, nv, nh = p.x_true.shape
        img = 8 * nv * nh * nt
        alg += 8 * nh * nt * nv * (nv + 1) // 2 + (11 if p.prior == "tv" else 9) * img
    total = 24 * iters
    res = {
        "workload": "24 uneven slices, 128x96x16 8c R4 .. 256x256x40 16c R10, TV and DFT alternating",
        "iterations_per_slice": iters,
        "batched_slice_iter_per_s": round(total / t_batch, 1),
        "plain_slice_iter_per_s": round(total / t_plain, 1),
        "speedup": round(t_plain / t_batch, 3),
        "batched_iter_per_s": round(iters / t_batch, 2),
        "algorithmic_GBps": round(alg * iters / t_batch / 1e9, 1),
        "hbm_frac": round(alg * iters / t_batch / 1e9 / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_batched_iteration": alg,
        "plans_s": round(t_plan, 2),
        "forms": sorted({int(p.flags) for p in plans}),
        "timing": f"median of {reps} runs, setup H'y included, host clock around device sync",
    }
    batch.close()
    return res


def unrolled_throughput(reps: int) -> dict:
    """K = 20 unrolled temporal-TV iterations on the 192x192x24, 12-coil, R=8
    workload with a checkpoint every 5: forward (cs_admm_forward_ckpt) and
    forward + backward (cs_admm_backward) passes per second, median of reps."""
    import torch
    from paper_1203_4587_amd import synthetic as S
    from paper_1203_4587_amd.api import Plan, to_device
    from paper_1203_4587_amd.autograd import Unrolled

    pr = S.CONFIGS["tv192_unrolled"]()
    plan = Plan(to_device(pr.coil), to_device(pr.mask, dtype=torch.uint8), pr.mu, prior="tv", mu_ratio=pr.rho)
    y = plan.apply_A(to_device(pr.x_true)) + to_device(pr.noise)
    un = Unrolled(plan, pr.iters, 5)
    g = torch.randn(plan.image_shape, dtype=torch.complex64, device="cuda")

    def fwd():
        un.forward_raw(y, pr.lam, pr.mu)

    def fb():
        un.forward_raw(y, pr.lam, pr.mu)
        un.backward_raw(g)

    res = {}
    for name, fn in (("forward", fwd), ("forward_backward", fb)):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        res[f"{name}_per_s"] = round(1.0 / _median(ts), 2)
        res[f"{name}_ms"] = round(1e3 * _median(ts), 3)
    # the same K with one segment: the forward keeps the whole tape and the
    # backward recomputes nothing (3 images per iteration of extra memory)
    un.close()
    un = Unrolled(plan, pr.iters, pr.iters)
    fb()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fb()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    res["forward_backward_full_tape_ms"] = round(1e3 * _median(ts), 3)
    nt, nv, nh = pr.x_true.shape
    res.update({
        "workload": "tv-192x192x24-12c R8, K=20 unrolled, checkpoint every 5",
        "backward_over_forward": round(res["forward_backward_ms"] / res["forward_ms"] - 1.0, 3),
        "factor_bytes": 8 * nh * nt * nv * (nv + 1) // 2,
    })
    un.close()
    plan.close()
    del y, g
    torch.cuda.empty_cache()
    # Algorithm 1 (temporal DFT) on the 192x192x40, 12-coil, R=10 workload
    pr = S.CONFIGS["dft192"]()
    plan = Plan(to_device(pr.coil), to_device(pr.mask, dtype=torch.uint8), pr.mu, prior="dft")
    y = plan.apply_A(to_device(pr.x_true)) + to_device(pr.noise)
    un = Unrolled(plan, 20, 5)
    g = torch.randn(plan.image_shape, dtype=torch.complex64, device="cuda")
    dres = {}
    for name, fn in (("forward", lambda: un.forward_raw(y, pr.lam, pr.mu)),
                     ("forward_backward", lambda: (un.forward_raw(y, pr.lam, pr.mu), un.backward_raw(g)))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        dres[f"{name}_ms"] = round(1e3 * _median(ts), 3)
    dres["workload"] = "dft-192x192x40-12c R10, K=20 unrolled, checkpoint every 5"
    res["dft"] = dres
    un.close()
    plan.close()
    return res


READ_STREAM_BLOCKS = (2048, 4096, 8192, 16384)


def stream_context(achieved) -> dict:
    """Context for the roofline fraction, which stays against the published
    peak: the rate of a plain torch device-to-device copy of 1 GiB (bytes
    read + written), and the library's pure read stream (cs_read_stream) over
    2 GiB at each grid of READ_STREAM_BLOCKS, the best of which is the read
    rate this chip sustains in practice.  Both are timed with torch events on
    the current stream, mean of 5 launches after a warm-up."""
    import torch
    from paper_1203_4587_amd.api import read_stream

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    copy = 2 * a.numel() * 4 / timed(lambda: b.copy_(a)) / 1e9
    del a, b
    buf = torch.zeros(2 ** 29, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    nbytes = buf.numel() * 4
    rates = {g: nbytes / timed(lambda: read_stream(buf, sink, blocks=g)) / 1e9 for g in READ_STREAM_BLOCKS}
    del buf, sink
    torch.cuda.empty_cache()
    best = max(rates, key=rates.get)
    out = {"device_copy_GBps": round(copy, 1),
           "read_stream_GBps": round(rates[best], 1),
           "read_stream_blocks": best,
           "read_stream_GBps_by_blocks": {str(g): round(r, 1) for g, r in rates.items()}}
    if achieved:
        out["frac_of_read_stream"] = round(achieved / rates[best], 4)
    return out


def same_bytes_copy(nbytes: int, reps: int = 50) -> dict:
    """A plain device copy moving nbytes in all (nbytes / 2 read, nbytes / 2
    written), each copy between its own pair of HIP events on the current
    stream, as the library times each launch: the rate a one-shot kernel of
    that size reaches when it does nothing but move its bytes."""
    import torch
    n = max(nbytes // 8, 1)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    del a, b
    us = _median(ts)
    return {"us_median": round(us, 2), "us_best": round(min(ts), 2), "GBps": round(8 * n / (us * 1e-6) / 1e9, 1)}


def step_rows(plan, problem, y, t_plan: float, prior: str) -> dict:
    """Per-step figures beside the iteration: the SENSE forward and adjoint
    passes (torch events on the stream they run on, mean of 20 calls), the
    plan build (host clock), and one objective evaluation (HIP events the
    library records around it during a traced solve)."""
    import torch
    nt, nv, nh = problem.x_true.shape
    nc = problem.coil.shape[0]
    m_rows = int(problem.mask.astype(bool).sum())           # sampled (frame, ky) rows
    img, coil_b = 8 * nt * nv * nh, 8 * nc * nv * nh
    sampled = 8 * m_rows * nc * nh                           # sampled rows of y, all coils

    def event_us(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e3 / reps

    def row(us, nbytes, what):
        gbs = nbytes / (us * 1e-6) / 1e9
        return {"us": round(us, 2), "algorithmic_bytes": nbytes, "bytes": what, "GBps": round(gbs, 1),
                "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}

    x = plan.apply_AH(y)
    yk = torch.empty_like(y)
    xo = torch.empty_like(x)
    a_us = event_us(lambda: plan.apply_A(x, out=yk))
    ah_us = event_us(lambda: plan.apply_AH(y, out=xo))
    rows = {
        "apply_A": row(a_us, img + coil_b + 8 * nt * nc * nv * nh,
                       "reads x and the coil maps, writes every k-space row (unsampled rows as zeros)"),
        "apply_AH": row(ah_us, sampled + coil_b + img, "reads the sampled rows of y and the coil maps, writes x"),
    }
    gj_flops = 8.0 * nv ** 3 * nh * nt
    rows["plan"] = {"s": round(t_plan, 4), "fp64_gauss_jordan_flops": gj_flops,
                    "fp64_TFLOPs_over_plan": round(gj_flops / t_plan / 1e12, 2),
                    "note": "whole plan build (Gram assembly, FP64 Gauss-Jordan inverse, packing) on the host clock"}
    plan.kernel_timing(True)
    plan.solve(y, problem.lam, 20, trace=True)
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.kernel_timing(False)
    n, ms = kt.get("objective", (0, 0.0))
    nf, fms = kt.get("frame_finish", (0, 0.0))
    if n and prior == "frame":
        # an evaluation is the pass completing w and d (reads x~, u, v, d;
        # writes w, d: 10 images) plus the objective itself
        rows["objective"] = row(ms * 1e3 / n + (fms * 1e3 / nf if nf else 0.0),
                                3 * img + coil_b + sampled + (10 * img if nf else 0),
                                "completes w and d (reads x~, u, v, d; writes w, d), then reads the coefficients "
                                "w (2 nt frames), x = Psi' w, the coil maps and the hybrid-space data")
    elif n:
        rows["objective"] = row(ms * 1e3 / n, img + coil_b + sampled,
                                "reads x, the coil maps and the hybrid-space data")
    return rows


def eigen_form(plan, problem, coil, mask, y, prior: str, steps: int, workload: str) -> dict:
    """The paper's own factor form (CS_FLAG_EIGEN: U diag(1/(mu + e)) U' per
    block) on the same workload: plan build, x-update rate against HBM peak,
    iteration rate, and what it saves, a refactor of the packed inverse when
    mu changes, expressed as the iterations per mu value below which it wins."""
    import torch
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    nt, nv, nh = problem.x_true.shape
    lam, mu = problem.lam, problem.mu

    def clock(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    out = {}
    t0 = time.perf_counter()
    eig = Plan(coil, mask, mu, prior=prior, mu_ratio=problem.rho, flags=_lib.CS_FLAG_EIGEN)
    torch.cuda.synchronize()
    out["plan_s"] = round(time.perf_counter() - t0, 3)
    eig.solve(y, lam, 5)
    eig_s = clock(lambda: eig.solve(y, lam, steps))
    eig.kernel_timing(True)
    eig.solve(y, lam, steps)
    torch.cuda.synchronize()
    xl, xms = eig.kernel_times().get("x_update", (0, 0.0))
    eig.kernel_timing(False)
    # per block: U' and U (n^2 complex64 each), e (n float); plus the right-hand
    # side and output traffic of the packed form's x-update
    nblk = nt * nh
    img = 8 * nv * nh * nt
    rhs = (5 if prior == "tv" else 3) * img
    alg = nblk * (2 * 8 * nv * nv + 4 * nv) + rhs
    us = xms / max(xl, 1) * 1e3
    gbs = alg / (us * 1e-6) / 1e9 if xl else None
    out.update({"iter_per_s": round(steps / eig_s, 2), "x_update_us": round(us, 2),
                "x_update_algorithmic_bytes": alg,
                "x_update_GBps": round(gbs, 1) if gbs else None,
                "x_update_hbm_frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None,
                "x_update_kernel": f"k_xupdate_{'eigen2' if nv % 2 == 0 else 'eigen'}",
                "x_update_traffic": measured_traffic(f"x_update_{'eigen2' if nv % 2 == 0 else 'eigen'}", workload,
                                                     1, eigen_source_sha),
                "plan_bytes": int(eig.nbytes)})
    # a mu change on the eigen plan costs nothing; on the packed plan it refactors
    eig_mu = clock(lambda: eig.solve(y, lam, steps, mu=mu * 1.5))
    eig.close()
    torch.cuda.empty_cache()
    packed_s = clock(lambda: plan.solve(y, lam, steps))
    refactor_s = clock(lambda: plan.solve(y, lam, 0, mu=mu * 1.5)) - clock(lambda: plan.solve(y, lam, 0, mu=mu * 1.5))
    plan.solve(y, lam, 0, mu=mu)  # back to the plan's mu (refactors again)
    torch.cuda.synchronize()
    per_iter_extra = (eig_s - packed_s) / steps
    out.update({"solve_at_new_mu_s": round(eig_mu, 5), "packed_refactor_s": round(refactor_s, 5),
                "breakeven_iterations_per_mu": round(refactor_s / per_iter_extra, 1) if per_iter_extra > 0 else None})
    return out


# block sizes of the x-update sweep: (nv, nh, nt), each factor at least twice
# the 256 MB last-level cache so that every launch streams it from HBM
XU_SWEEP = [(64, 512, 64), (128, 256, 64), (192, 192, 40), (256, 256, 32), (384, 128, 16), (512, 64, 16)]


def xu_sweep() -> dict:
    """The x-update's rate across block sizes n_v: a 10-iteration temporal-DFT
    solve (4 coils, R = 4, seeded synthetic data) per size with HIP events
    around every launch; algorithmic bytes = packed factor + 3 images (reads
    H'y and u, writes z), as in the roofline object."""
    import torch
    from paper_1203_4587_amd import synthetic as S
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan, to_device
    out = []
    for nv, nh, nt in XU_SWEEP:
        pr = S.make_problem(nv, nh, nt, 4, 4, 8, "dft", "periodic", 3000 + nv, name=f"xu-{nv}")
        plan = Plan(to_device(pr.coil), to_device(pr.mask, dtype=torch.uint8), pr.mu, prior="dft")
        y = plan.apply_A(to_device(pr.x_true)) + to_device(pr.noise)
        plan.solve(y, pr.lam, 5)
        plan.kernel_timing(True)
        plan.solve(y, pr.lam, 10)
        torch.cuda.synchronize()
        n, ms = plan.kernel_times().get("x_update", (0, 0.0))
        plan.kernel_timing(False)
        f = plan.flags
        form = ("rows" if nv % 2 else "wave2" if nv % 64 == 0 and (nv // 2) % 64 and not (f & _lib.CS_FLAG_XU_GROUP)
                else "wave" if (nv // 2) % 64 == 0 and not (f & _lib.CS_FLAG_XU_GROUP) else "pairs")
        nbytes = 8 * nh * nt * nv * (nv + 1) // 2 + 3 * 8 * nt * nv * nh
        us = ms * 1e3 / max(n, 1)
        out.append({"nv": nv, "nh": nh, "nt": nt, "blocks": nh * nt, "form": form, "launches": n,
                    "us": round(us, 2), "algorithmic_bytes": nbytes, "GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                    "hbm_frac": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
        log(f"x-update sweep nv={nv}: {out[-1]['us']} us, {out[-1]['GBps']} GB/s ({form})")
        plan.close()
        del y
        torch.cuda.empty_cache()
    return {"xu_sweep": out, "peak_GBps": HBM_PEAK_GBS}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed ADMM iterations")
    ap.add_argument("--warmup", type=int, default=10, help="untimed ADMM iterations before the timed solve")
    ap.add_argument("--repeats", type=int, default=10,
                    help="further timed solves of --steps iterations, reported as min and median")
    ap.add_argument("--workload", default="tv256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=16)
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--no-delta", action="store_true", help="skip the solve to Delta(k) < 1e-3")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--batched-iters", type=int, default=100, help="iterations per slice in that comparison")
    ap.add_argument("--no-unrolled", action="store_true", help="skip the differentiated-solve measurement")
    ap.add_argument("--unrolled-reps", type=int, default=10, help="timed forward+backward passes")
    ap.add_argument("--no-tune", action="store_true", help="time the default form instead of the tuned one")
    ap.add_argument("--no-eigen", action="store_true", help="skip the eigen-form (any-mu) factor measurement")
    ap.add_argument("--xu-sweep", action="store_true",
                    help="only measure the x-update across block sizes n_v = 64 .. 512 and print that JSON object")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the per-step figures (SENSE passes, plan, objective monitor)")
    ap.add_argument("--xu-form", choices=["wave", "group"], default=None,
                    help="force an x-update form (implies --no-tune; used for per-kernel counter passes)")
    ap.add_argument("--column-resident", action="store_true",
                    help="one launch for all iterations (a workgroup per readout column) instead of two "
                         "launches per iteration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the benchmark runs the reconstruction on one "
              "GPU (readout columns are independent ADMM problems, so more GPUs would each take a column range "
              "or whole slices)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1203_4587_amd import synthetic as S
    from paper_1203_4587_amd.api import Plan, to_device

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.xu_sweep:
        print(json.dumps(xu_sweep()), flush=True)
        return 0
    wl = WORKLOADS[args.workload]
    problem = S.CONFIGS[wl.get("config", args.workload)]()
    nt, nv, nh = problem.x_true.shape
    nc = problem.coil.shape[0]

    coil = to_device(problem.coil)
    mask = to_device(problem.mask, dtype=torch.uint8)
    t0 = time.perf_counter()
    from paper_1203_4587_amd import _lib
    flags = _lib.CS_FLAG_COLUMN_RESIDENT if args.column_resident else 0
    if args.xu_form:
        args.no_tune = True
        flags |= _lib.CS_FLAG_XU_WAVE if args.xu_form == "wave" else _lib.CS_FLAG_XU_GROUP
    plan = Plan(coil, mask, problem.mu, prior=wl["prior"], mu_ratio=problem.rho, flags=flags)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    # synthetic measured data y = H x_true + noise, formed on the device
    y = plan.apply_A(to_device(problem.x_true)) + to_device(problem.noise)
    torch.cuda.synchronize()
    log(f"plan: {t_plan:.2f} s, {plan.nbytes / 2**30:.2f} GiB on device")

    if args.calib_copy_mib:
        n = args.calib_copy_mib * 2**20 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    tuned = None
    if not args.column_resident and not args.no_tune:
        # the library's autotuner picks the execution form (x-update form, graph
        # replay, column groups on concurrent branches) on this data, untimed
        tuned = plan.tune(y, problem.lam, iters=10)
        log(f"tuned form: flags {tuned['flags']} of {len(tuned['candidates'])} candidates")
    if args.warmup:
        plan.solve(y, problem.lam, args.warmup)
    x = torch.empty(plan.image_shape, dtype=torch.complex64, device="cuda")
    # one untimed solve of the timed length: the graph form caches one recorded
    # loop per iteration count, so this records the loop the timed solve replays
    plan.solve(y, problem.lam, args.steps, out=x)
    torch.cuda.synchronize()

    # timed region: one solve of --steps iterations in the chosen form
    t0 = time.perf_counter()
    plan.solve(y, problem.lam, args.steps, out=x)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # the same solve repeated (the paper reports the fastest of 10 runs, Sec. V)
    rep_s = []
    for _ in range(args.repeats):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.solve(y, problem.lam, args.steps, out=x)
        torch.cuda.synchronize()
        rep_s.append(time.perf_counter() - t)

    # second timed solve of the same length with HIP events around every
    # launch (single-stream phase form, since events cannot sit inside a
    # replayed graph): per-kernel durations for the roofline
    plan.kernel_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.solve(y, problem.lam, args.steps, out=x)
    torch.cuda.synchronize()
    elapsed_events = time.perf_counter() - t1
    ktimes = plan.kernel_times()
    plan.kernel_timing(False)

    value = args.steps / elapsed
    npix = nv * nh
    img_bytes = 8 * npix * nt
    factor_bytes = 8 * nh * nt * nv * (nv + 1) // 2
    if wl["prior"] == "tv":
        x_bytes = factor_bytes + 5 * img_bytes          # reads H'y, m, d2; writes x, d2
        t_bytes = 6 * img_bytes - 2 * 8 * npix          # reads m, d1, x, d2; writes m, d1 (d1: nt-1 frames)
        tkind = "tv_step"
    elif wl["prior"] == "dft":
        x_bytes = factor_bytes + 3 * img_bytes          # reads H'y, u; writes z
        t_bytes = 6 * img_bytes                         # reads z, d, v; writes d, v, u
        tkind = "dft_step"
    else:
        x_bytes = factor_bytes + 3 * img_bytes          # reads H'y, u; writes x~
        t_bytes = 11 * img_bytes                        # reads x~, u, v, d (2 nt frames each); writes v, d, u
        tkind = "dft_step"
    if "column_solve" in ktimes:
        # one launch runs every iteration: temporal step + x-update per column
        kind = "column_solve"
        launches, ms = ktimes[kind]
        alg_bytes = (x_bytes + t_bytes) * args.steps
        kdesc = ("column_solve (one launch for all iterations; per readout column: temporal step, then "
                 "x-update streaming the packed Hermitian (mu I + G)^-1 of each frame)")
    else:
        kind = "x_update"
        launches, ms = ktimes.get(kind, (0, 0.0))
        alg_bytes = x_bytes
        kdesc = "x_update (packed Hermitian (mu I + G)^-1 per column and frame)"
    avg_s = ms / max(launches, 1) / 1e3
    achieved = alg_bytes / avg_s / 1e9 if launches else None
    tl, tms = ktimes.get(tkind, (0, 0.0))
    xl, xms = ktimes.get("x_update", (0, 0.0))
    if kind == "x_update":
        # which x-update kernel ran (the forms move the same bytes; counters are per kernel)
        f = plan.flags
        sha_fn = None
        if nv % 2:
            family = "rows"
        elif not (f & _lib.CS_FLAG_XU_GROUP) and nv % 64 == 0 and (nv // 2) % 64:
            family, sha_fn = "wave2", wave2_source_sha   # two blocks per wave (nv = 64, 192)
        elif not (f & _lib.CS_FLAG_XU_GROUP) and ((f & _lib.CS_FLAG_XU_WAVE) or (nv // 2) % 64 == 0):
            family = "wave"
        else:
            family = "pairs"
        kdesc += f"; kernel k_xupdate_{family}"
        traffic = measured_traffic(f"x_update_{family}", args.workload, args.steps, sha_fn)
    else:
        traffic = measured_traffic(kind, args.workload, args.steps)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64",
        "data": "synthetic",
        "config": {
            "workload": wl["name"], "prior": wl["prior"], "nv": nv, "nh": nh, "nt": nt, "nc": nc,
            "accel": int(round(nv / max(int(problem.mask[0].sum()), 1))), "lambda": problem.lam,
            "mu": problem.mu, "mu_ratio": problem.rho, "iterations_per_solve": args.steps,
            "parallelism": "none",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kdesc,
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_us": round(avg_s * 1e6, 2),
            "launches": launches,
        },
        "kernels": {
            "iteration_us": round(avg_s * 1e6 / (args.steps if kind == "column_solve" else 1), 2),
            "x_update_us": round(xms / max(xl, 1) * 1e3, 2) if xl else None,
            f"{tkind}_us": round(tms / max(tl, 1) * 1e3, 2) if tl else None,
            "factor_bytes_per_iteration": factor_bytes,
            "iteration_algorithmic_bytes": x_bytes + t_bytes,
            "iteration_algorithmic_GBps": round((x_bytes + t_bytes) * value / 1e9, 1),
        },
        "plan_s": round(t_plan, 3),
        "repeats": {
            "solves": len(rep_s), "iterations_each": args.steps,
            "iter_per_s_best": round(args.steps / min(rep_s), 2) if rep_s else None,
            "iter_per_s_median": round(args.steps / _median(rep_s), 2) if rep_s else None,
            "ms_per_step_min": round(1e3 * min(rep_s) / args.steps, 4) if rep_s else None,
            "ms_per_step_median": round(1e3 * _median(rep_s) / args.steps, 4) if rep_s else None,
            "timing": "host clock around each solve, device synchronised on both sides; graph replays",
        },
        "form": {
            "flags": int(plan.flags),
            "tuned": tuned is not None,
            "candidates_ms_per_iter": [[int(f), round(m, 4)] for f, m in tuned["candidates"]] if tuned else None,
            "event_timed_iter_per_s": round(args.steps / elapsed_events, 2),
        },
    }
    line["roofline"].update(stream_context(achieved))
    if tl:
        # the temporal step against a device copy of the same bytes, both
        # event-timed per launch
        t_us = tms / tl * 1e3
        cp = same_bytes_copy(t_bytes)
        line["kernels"][f"{tkind}_algorithmic_bytes"] = t_bytes
        line["kernels"][f"{tkind}_GBps"] = round(t_bytes / (t_us * 1e-6) / 1e9, 1)
        line["kernels"][f"{tkind}_same_bytes_copy"] = cp
        line["kernels"][f"{tkind}_frac_of_copy"] = round(cp["us_median"] / t_us, 3)
    if not args.no_rows:
        line["rows"] = step_rows(plan, problem, y, t_plan, wl["prior"])
    # the paper's stopping rule: iterate until Delta(k) < 1e-3 (checked every 5
    # iterations, J on the device), timed like the fixed-count solve
    if not args.no_delta:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, k_done, d_last = plan.solve_until(y, problem.lam, 1000, tol=1e-3, check_every=5, out=x)
        torch.cuda.synchronize()
        t_delta = time.perf_counter() - t2
        line["to_delta"] = {"tol": 1e-3, "check_every": 5, "iterations": k_done, "delta": d_last,
                            "seconds": round(t_delta, 5), "iter_per_s": round(k_done / t_delta, 2)}
    if not args.no_eigen and not args.column_resident:
        log("eigen-form factor ...")
        line["eigen"] = eigen_form(plan, problem, coil, mask, y, wl["prior"], args.steps, args.workload)
    plan.close()
    del x, y
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched vs plain: 24 uneven slices ...")
        line["batched"] = batched_vs_plain(args.batched_iters)
        torch.cuda.empty_cache()
    if not args.no_unrolled:
        log("differentiated unrolled solve ...")
        line["unrolled"] = unrolled_throughput(args.unrolled_reps)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a column sample ...")
        line["cpu_baseline"] = cpu_baseline(problem, args.cpu_cols, args.cpu_iters)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
