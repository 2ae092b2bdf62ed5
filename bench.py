"""Benchmark of the Hopf evaluation hot path on one MI355X.

Workload (default): n = 1024, dense SPD A = Q diag(s) Q^T (Q Haar, s log-uniform [0.1, 10]),
H = ||p||_2 + sum w_i |p_i| (w ~ U(0.5, 2)), 2^16 points x ~ N(0, 4I), t ~ U(0.05, 3), FP32
inputs, BF16 MFMA products refined by FP64-exact anchor products.  One step = the whole path
for one batch: problem set-up (FP64 inverse of A + lambda I on the device), the split-Bregman
evaluation of every point (phi, grad phi, dphi/dt) and the release of the problem.

Prints one JSON line (rank 0) with the throughput, the roofline of the dominant kernel
(measured with HIP events on the launch stream), the accuracy against the FP64 oracle on a
sample, and the oracle's own rate on a bounded sample of the same workload (CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 MFMA
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 (matrix)
METRIC = "Hopf point-evals/sec (φ+∇φ) at n=1024, 1e-6 rel vs FP64; % roofline"

# HBM traffic of the dominant kernel on the default workload, from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE; the profiles/ summary of the n=1024 workload), each scaled by what the
# counter reads for a plain 256 MiB device copy.  Valid only for the kernel source it was measured
# on (hash of TRAFFIC_SOURCES); reported as null otherwise.
TRAFFIC_SOURCES = ("dense_rs.hip", "dense_shared.hpp", "common.hpp")
TRAFFIC = {"source_sha256": "bb3807aefc5e4b2402f105d245d2e27325dbf39aff34fc71505e1ab5037999f9",
           "read_bytes": 121.391e9, "write_bytes": 10.149e9, "precision": "bf16_refined", "npts": 1 << 16,
           "tol": 1e-12}


def measured_traffic(precision, npts, tol):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1605_01799_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if (h.hexdigest() != TRAFFIC["source_sha256"] or precision != TRAFFIC["precision"]
            or npts != TRAFFIC["npts"] or tol != TRAFFIC["tol"] or os.environ.get("HOPF_RS", "1") == "0"
            or os.environ.get("HOPF_RS_ANCHOR_EVERY", "24") != "24"):
        return None
    return TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"]


# The same for the tile kernel of the n=256 union workload (c5; its profiles/ summary), valid for
# the sources, the tuned launch shapes and the point count and tolerance it was measured on.
C5_TRAFFIC = {"sources": ("dense.hip", "dense_shared.hpp", "common.hpp", "api.hip", "tune_table.inc"),
              "source_sha256": "8a0b7392b9ed08e2772106bf0dbf65dc3065980c5c457d60dffa9b9d54fda650",
              "read_bytes": 26.721e9, "write_bytes": 173.840e9, "npts": 1 << 18, "tol": 1e-12}


def measured_traffic_c5(npts, tol):
    import hashlib
    h = hashlib.sha256()
    for f in C5_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, "paper_1605_01799_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if (h.hexdigest() != C5_TRAFFIC["source_sha256"] or npts != C5_TRAFFIC["npts"] or tol != C5_TRAFFIC["tol"]
            or "HOPF_DENSE_VARIANT" in os.environ or os.environ.get("HOPF_ANCHOR_EVERY", "32") != "32"):
        return None
    return C5_TRAFFIC["read_bytes"] + C5_TRAFFIC["write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16_refined", choices=["bf16_refined", "f32"])
    ap.add_argument("--npts", type=int, default=1 << 16)
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the BF16-only error measurement (thousands of small torch launches: "
                         "left out of profiled runs)")
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="most points of the CPU baseline's stratified sample (it is sized to ~15 s)")
    ap.add_argument("--acc-sample", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--deterministic", action="store_true",
                    help="the library's deterministic mode (fixed chunk schedule; hopf_set_deterministic); "
                         "the line's config then says so")
    ap.add_argument("--workload", default="c3",
                    choices=["c3", "c1s", "c2", "c4", "c5", "c2wl2", "pd16", "pa16", "t5n16", "lc16", "c3wl2"],
                    help="c3 (default): the metric workload.  Other hot-path workloads, one JSON line "
                         "each: c1s = n=8 FP64 diagonal path at 2^24 points (HBM roofline), c2 = n=64 "
                         "FP32 dense at 2^20 points, c4 = the ragged batch of 4096 problems (n log-uniform "
                         "in [4, 2048], union of 8 ellipsoids, FP32; generation takes minutes on the host: "
                         "use --steps 2 --warmup 1), c5 = n=256 union of 4 ellipsoids, forward + backward; "
                         "c2wl2 = c2 with H = sqrt(<p, diag(w) p>); pd16 = the paper's timing-table setting "
                         "for that H at n=16 (J = 1/2 <y, D^-1 y>, FP64, tol 1e-8); pa16 = the same for "
                         "H = sqrt(<p, HA p>), HA = I + 1 1^T (FP32, the wave-local kernel in HA's eigenbasis); "
                         "t5n16 = the paper's Table 5 workload, J = 1/2 |y|_1^2, H = |p|_inf, n=16, FP64, tol 1e-8; "
                         "lc16 = the time-dependent H of linear controls (diagonal drift and inputs, box controls), "
                         "n=16, FP64, tol 1e-20; c3wl2 = the n=1024 workload with H = sqrt(<p, diag(w) p>) (the "
                         "tile kernel's multiplier solves), BF16 refined")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="only run a plain device copy of 256 MiB (x5): the reference kernel for the "
                         "scale of the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_calibrate():
    import torch
    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 5}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only (the workload is one GPU's share of the points); "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.copy_calibrate:
        copy_calibrate()
        return
    global SKIP_CPU
    SKIP_CPU = a.no_cpu
    if a.deterministic:
        from paper_1605_01799_amd import hopf as H
        H.set_deterministic(True)
    if a.workload != "c3":
        bench_other(a)
        return
    import torch
    from paper_1605_01799_amd import hopf as H
    from paper_1605_01799_amd import workloads as W

    tol = a.tol if a.tol is not None else (1e-12 if a.precision == "bf16_refined" else 1e-10)
    p = W.round_inputs(W.workload3(npts=a.npts))
    n, npts = p.n, p.npts
    dev = torch.device("cuda:0")
    x = torch.from_numpy(p.x).to(dev)
    t = torch.from_numpy(p.t).to(dev)
    stream = torch.cuda.current_stream()
    out = dict(phi=torch.empty(npts, device=dev), grad=torch.empty(npts, n, device=dev),
               dphidt=torch.empty(npts, device=dev), iters=torch.empty(npts, dtype=torch.int32, device=dev),
               kstar=torch.empty(npts, dtype=torch.int32, device=dev))
    kw = dict(hkind="l2_wl1", w=p.w, tol=tol, max_iter=20000, precision=a.precision)

    def step(ev=None):
        prob = H.Problem(p.A, **kw)
        if ev is not None:
            ev[0].record(stream)
        prob.eval(x, t, out=out)
        if ev is not None:
            ev[1].record(stream)
        del prob          # hopf_problem_destroy
        return

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    eval_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    value = npts / (ms_per_step / 1e3)

    iters = out["iters"].cpu().numpy()
    if np.any(iters <= 0):
        print("warning: %d points did not converge" % int(np.sum(iters <= 0)), file=sys.stderr)
    flops = float(np.sum(np.maximum(iters, 0)).astype(np.float64) * 2.0 * n * n)
    achieved = flops / (eval_ms / 1e3) / 1e12
    peak = BF16_PEAK_TFLOPS if a.precision == "bf16_refined" else FP32_PEAK_TFLOPS

    rec = {
        "metric": METRIC, "value": value, "unit": "point-evals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16" if a.precision == "bf16_refined" else "f32",
        "data": "synthetic",
        "config": {"workload": "n=1024 dense SPD A, H=l2+weighted l1, 2^16 points x~N(0,4I), t~U(0.05,3), "
                               "FP32 inputs, split Bregman lambda=1; step = FP64 set-up + evaluation",
                   "n": n, "npts": npts, "tol": tol, "precision": a.precision,
                   "products": "BF16 MFMA on increments + exact anchors (int8 MFMA on integer slices)"
                   if a.precision == "bf16_refined"
                   else "FP32 MFMA"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(a.precision, npts, tol), "traffic_unit": "HBM bytes read + written per launch",
                     "kernel": ("dense_rs_kernel<8, bf16x4> (on-chip column state; one launch per step)"
                                if a.precision == "bf16_refined" and os.environ.get("HOPF_RS", "1") != "0"
                                else "dense_kernel (one launch per step)"),
                     "algorithmic": "sum over points of iterations x 2 n^2 FLOP",
                     "flop_per_launch": flops, "launch_ms": eval_ms},
        "eval_only": {"ms": eval_ms, "value": npts / (eval_ms / 1e3)},
        "iterations": {"mean": float(iters.mean()), "p50": float(np.median(iters)),
                       "p99": float(np.percentile(iters, 99)), "max": int(iters.max())},
    }

    # accuracy on a sample against the FP64 oracle (tight tolerance), and the CPU baseline
    try:
        import oracle
        oracle.build(force=not oracle.available())
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample, npts), replace=False))
        xs = p.x[idx].astype(np.float64)
        ts = p.t[idx].astype(np.float64)
        threads = max(1, min(host_info()["affinity"], CPU_SHARE))
        ref = oracle.oracle_eval(p.A, xs, ts, "l2_wl1", w=p.w, tol=1e-28, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ph = out["phi"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        ef = np.abs(ph - ref["phi"]) / np.maximum(np.abs(ref["phi"]), 1)
        rec["accuracy"] = {"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()),
                           "max_rel_err_phi": float(ef.max()), "bound": 1e-6,
                           "ok": bool(ep.max() <= 1e-6 and ef.max() <= 1e-6)}
        if a.precision == "bf16_refined" and not a.no_bf16:
            rec["bf16_only"] = bf16_only_error(p, idx, ref["grad"], dev)
        if not a.no_cpu:
            rec["cpu_baseline"] = cpu_baseline(
                lambda idx, nt: oracle.oracle_eval(p.A, p.x[idx].astype(np.float64), p.t[idx].astype(np.float64),
                                                   "l2_wl1", w=p.w, tol=tol, nthreads=nt),
                p.t, a.cpu_sample, "same tol (%g), FP64 oracle (triangular solves, compensated sums)" % tol)
    except Exception as e:  # the oracle is test infrastructure; its absence only drops these fields
        rec["accuracy_error"] = str(e)
    if a.deterministic:
        rec.setdefault("config", {})["deterministic"] = True
    print(json.dumps(rec), flush=True)


def bf16_only_error(p, idx, ref_grad, dev, lam=1.0, iters=4000):
    """Error of the plain split-Bregman iteration with BF16 products alone (no exact anchors) on
    the accuracy sample, beside the a-priori kappa(A + lambda I) 2^-8: M and every right-hand
    side rounded to BF16, products accumulated and the state kept in FP32, run to its own fixed
    point.  A measurement of the precision form (torch operations on the GPU), not the solver."""
    import torch
    Ad = np.asarray(p.A, np.float64)
    n = Ad.shape[0]
    ev = np.linalg.eigvalsh(Ad)
    kappa = float((ev.max() + lam) / (ev.min() + lam))
    M = np.linalg.inv(Ad + lam * np.eye(n))
    Mb = torch.from_numpy(M).to(dev).to(torch.bfloat16).float()
    X = torch.from_numpy(p.x[idx].astype(np.float32)).to(dev).T.contiguous()      # n x m
    T = torch.from_numpy(p.t[idx].astype(np.float32)).to(dev)
    w = torch.from_numpy(np.asarray(p.w, np.float32)).to(dev)[:, None]
    th1 = w * (T / lam)[None, :]
    th2 = (T / lam)[None, :]

    def prox(z):  # H = |.|_2 + sum w_i |.|: shrink1 then shrink2
        s1 = z - torch.clamp(torch.maximum(z, -th1), max=th1)
        nz = torch.linalg.norm(s1, dim=0, keepdim=True)
        return s1 * torch.clamp(nz - th2, min=0) / torch.where(nz > 0, nz, torch.ones_like(nz))
    z = X.clone()
    for _ in range(iters):
        d = prox(z)
        r = X + lam * (2 * d - z)
        z = z - d + Mb @ r.to(torch.bfloat16).float()
    g = prox(z).T.cpu().numpy().astype(np.float64)
    e = np.linalg.norm(g - ref_grad, axis=1) / np.maximum(np.linalg.norm(ref_grad, axis=1), 1)
    return {"max_rel_err_grad": float(e.max()), "median_rel_err_grad": float(np.median(e)),
            "kappa_A_plus_lambda_I": kappa, "kappa_times_2^-8": kappa * 2.0 ** -8,
            "how": "plain iteration, %d passes, BF16-rounded M and right-hand sides, FP32 accumulation and state "
                   "(torch on the GPU), same %d points as accuracy" % (iters, len(idx))}


def timed_steps(step, steps, warmup):
    """Runs warmup + steps calls of step(ev); returns (ms per step by the host clock, mean ms
    between the events each step records around its dominant launch)."""
    import torch
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))


# host threads per GPU on the shared GPU hosts: the baseline uses at most this many
CPU_SHARE = 16
SKIP_CPU = False  # --no-cpu: no CPU baseline (sweeps and profiled runs)


def host_info():
    """CPU model, logical CPU count and the CPUs this process may run on."""
    import platform
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"cpu_model": model or platform.processor(), "nproc": os.cpu_count(), "affinity": aff}


def stratified(t, m):
    """m indices spread evenly over the points sorted by t (iteration counts follow t)."""
    order = np.argsort(np.asarray(t), kind="stable")
    pos = np.unique(np.linspace(0, len(order) - 1, max(1, m)).round().astype(int))
    return np.sort(order[pos])


def cpu_baseline(run, t, cap, what, budget_s=15.0, one_thread_pts=8):
    """The oracle's rate on the host: first one thread on a few stratified points, then all
    threads of the GPU's CPU share on a stratified sample sized to about budget_s seconds (at
    most cap points).  run(idx, nthreads) evaluates the oracle on the points idx."""
    if SKIP_CPU:
        return None
    info = host_info()
    threads = max(1, min(info["affinity"], CPU_SHARE))
    idx1 = stratified(t, min(one_thread_pts, len(t)))
    c0 = time.perf_counter()
    run(idx1, 1)
    rate1 = len(idx1) / (time.perf_counter() - c0)
    m = int(min(cap, len(t), max(threads, rate1 * threads * budget_s)))
    idx = stratified(t, m)
    c0 = time.perf_counter()
    run(idx, threads)
    rate = len(idx) / (time.perf_counter() - c0)
    return {"value": rate, "unit": "point-evals/s", "cores": threads, "kind": "oracle",
            "one_thread": rate1, **info,
            "sample": "%d points stratified by t (sized to ~%.0f s, at most %d), %s, %d threads (the GPU's "
                      "CPU share); one_thread: %d points on one thread" % (len(idx), budget_s, cap, what, threads,
                                                                           len(idx1))}


def bench_other(a):
    import torch
    from paper_1605_01799_amd import hopf as H
    from paper_1605_01799_amd import workloads as W
    import oracle
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    threads = max(1, min(host_info()["affinity"], CPU_SHARE))
    rec = {"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
           "unit": "point-evals/s"}

    if a.workload == "c1s":
        npts = a.npts if a.npts != 1 << 16 else 1 << 24
        p = W.workload_scaled_n8(npts)
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        prob = H.Problem(np.ones(p.n), diagonal=True, hkind="wl1", precision="f64", tol=1e-24, max_iter=500)
        out = dict(phi=torch.empty(npts, dtype=torch.float64, device=dev),
                   grad=torch.empty(npts, p.n, dtype=torch.float64, device=dev),
                   dphidt=torch.empty(npts, dtype=torch.float64, device=dev),
                   iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
        ms, kms = timed_steps(step, a.steps, a.warmup)
        per_point = 8 * p.n + 8 + 8 * p.n + 8 + 8 + 4 + 4   # x, t in; p, phi, dphidt, iters, kstar out
        achieved = npts * per_point / (kms / 1e3) / 1e9
        # the closed form of this workload (A = I, H = l1): p = sign(x) max(|x| - t, 0)
        g = out["grad"].cpu().numpy()
        pcf = np.sign(p.x) * np.maximum(np.abs(p.x) - p.t[:, None], 0)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(np.eye(p.n), p.x[idx], p.t[idx], "wl1", tol=1e-24,
                                                              max_iter=500, nthreads=nt),
                           p.t, 1 << 22, "same tol, FP64 oracle", one_thread_pts=1 << 14)
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=8 FP64 diagonal path; % HBM roofline",
                   value=npts / (ms / 1e3), steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f64",
                   config={"workload": "n=8, A=I, H=l1, %d points x~N(0,1), t~U(0.1,2), FP64, tol 1e-24, "
                                       "cap 500" % npts, "npts": npts},
                   roofline={"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                             "frac": achieved / 8000.0, "traffic": None, "kernel": "diag_kernel<double, 8>",
                             "algorithmic": "%d B per point (in and out)" % per_point, "launch_ms": kms},
                   accuracy={"max_abs_err_grad_vs_closed_form": float(np.abs(g - pcf).max()), "points": npts},
                   cpu_baseline=cpu)
    elif a.workload == "pd16":
        npts = a.npts if a.npts != 1 << 16 else 1 << 22
        p = W.workload_paper_d(16, npts, True)
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        tol = a.tol if a.tol is not None else 1e-8
        prob = H.Problem(np.diag(p.A).copy(), diagonal=True, hkind="wl2", w=p.w, precision="f64", tol=tol,
                         max_iter=20000)
        out = dict(phi=torch.empty(npts, dtype=torch.float64, device=dev),
                   grad=torch.empty(npts, p.n, dtype=torch.float64, device=dev),
                   dphidt=torch.empty(npts, dtype=torch.float64, device=dev),
                   iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
        ms, kms = timed_steps(step, a.steps, a.warmup)
        it = out["iters"].cpu().numpy()
        # split-Bregman work per point-iteration without the multiplier's Newton steps (a lower
        # bound on the FP64 operations): 3n (v), 2n (z), 4n (b), 6n (three norms)
        flops = float(np.sum(np.abs(it)).astype(np.float64) * 15.0 * p.n)
        achieved = flops / (kms / 1e3) / 1e12
        rng = np.random.default_rng(8)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample * 4, npts), replace=False))
        ref = oracle.oracle_eval(p.A, p.x[idx], p.t[idx], "wl2", w=p.w, tol=1e-28, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(p.A, p.x[idx], p.t[idx], "wl2", w=p.w, tol=tol,
                                                              max_iter=20000, nthreads=nt),
                           p.t, 1 << 20, "same tol, FP64 oracle", one_thread_pts=1 << 12)
        value = npts / (ms / 1e3)
        paper_s = 6.64e-06   # Table 4, H = ||.||_D, n = 16: seconds per evaluation on one laptop core
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=16 FP64 diagonal path, H=sqrt(<p,Dp>); "
                          "% FP64 vector roofline",
                   value=value, steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f64",
                   vs_baseline=value * paper_s,
                   config={"workload": "paper timing-table setting: n=16, D_ii = 1+(i-1)/15, J = 1/2 <y, D^-1 y>, "
                                       "H = sqrt(<p, D p>), %d points x~U[-10,10]^16, t~U(0,10], FP64, tol %g"
                                       % (npts, tol), "npts": npts},
                   roofline={"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                             "frac": achieved / 78.6, "traffic": None, "kernel": "diag_kernel<double, 16>",
                             "algorithmic": "sum over points of iterations x 15 n FP64 operations (the "
                                            "split-Bregman updates; the projection's Newton steps not counted, "
                                            "so a lower bound)", "launch_ms": kms},
                   iterations={"mean": float(np.abs(it).mean()), "capped": int(np.sum(it == -2))},
                   accuracy={"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()), "bound": None,
                             "note": "against the converged oracle (tol 1e-28); the paper's stop rule "
                                     "(squared norms <= 1e-8) itself leaves errors of this size"},
                   paper={"seconds_per_eval": paper_s, "hardware": "one core of an i5-5300U (Table 4)",
                          "note": "vs_baseline = value / (1 / seconds_per_eval): another machine, context only"},
                   cpu_baseline=cpu)
    elif a.workload == "c3wl2":
        npts = a.npts
        p = W.round_inputs(W.workload3_wl2(npts))
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        tol = a.tol if a.tol is not None else 1e-12
        prob = H.Problem(p.A, hkind="wl2", w=p.w, precision="bf16_refined", tol=tol, max_iter=20000)
        out = dict(phi=torch.empty(npts, device=dev), grad=torch.empty(npts, p.n, device=dev),
                   dphidt=torch.empty(npts, device=dev), iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
        for _ in range(a.warmup):
            step(None)
        torch.cuda.synchronize()
        prob.iterations(reset=True)
        ms, kms = timed_steps(step, a.steps, 0)
        passes = prob.iterations(reset=True) / a.steps   # counted on the device
        flops = float(passes) * 2.0 * p.n * p.n
        achieved = flops / (kms / 1e3) / 1e12
        it = out["iters"].cpu().numpy()
        idx = stratified(p.t, min(a.acc_sample, npts))
        ref = oracle.oracle_eval(p.A, p.x[idx].astype(np.float64), p.t[idx].astype(np.float64), "wl2", w=p.w,
                                 tol=1e-26, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        ef = np.abs(out["phi"].cpu().numpy()[idx] - ref["phi"]) / np.maximum(np.abs(ref["phi"]), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(p.A, p.x[idx].astype(np.float64),
                                                              p.t[idx].astype(np.float64), "wl2", w=p.w, tol=tol,
                                                              nthreads=nt),
                           p.t, 4096, "same tol, FP64 oracle")
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=1024 dense, H=sqrt(<p,Dp>), BF16 refined; % BF16 MFMA "
                          "roofline",
                   value=npts / (ms / 1e3), steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="bf16",
                   config={"workload": "n=1024 dense SPD A (workload 3's), H=sqrt(<p, diag(w) p>), %d points "
                                       "x~N(0,4I), t~U(0.05,3), FP32 inputs, tol %g" % (npts, tol), "npts": npts},
                   roofline={"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                             "kernel": "dense_kernel<1, 2, 2, 2, 4> (tile kernel; multiplier phase per pass)",
                             "algorithmic": "passes counted on the device x 2 n^2 FLOP (the multiplier's Newton "
                                            "sweeps not counted)", "launch_ms": kms},
                   iterations={"mean": float(np.abs(it).mean()), "passes_per_point": float(passes) / npts},
                   accuracy={"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()),
                             "max_rel_err_phi": float(ef.max()), "bound": 1e-6},
                   cpu_baseline=cpu)
    elif a.workload == "lc16":
        npts = a.npts if a.npts != 1 << 16 else 1 << 22
        p = W.workload_linear_control(16, npts)
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        tol = a.tol if a.tol is not None else 1e-20
        adiag = np.diag(p.A).copy()
        prob = H.Problem(adiag, diagonal=True, hkind="linctrl", w=p.w, drift=p.drift, precision="f64", tol=tol,
                         max_iter=20000)
        out = dict(phi=torch.empty(npts, dtype=torch.float64, device=dev),
                   grad=torch.empty(npts, p.n, dtype=torch.float64, device=dev),
                   dphidt=torch.empty(npts, dtype=torch.float64, device=dev),
                   iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
        ms, kms = timed_steps(step, a.steps, a.warmup)
        it = out["iters"].cpu().numpy()
        # per point-iteration: 3n (v), 4n (z and shrink), 2n (b), 6n (three norms) FP64 operations
        flops = float(np.sum(np.abs(it)).astype(np.float64) * 15.0 * p.n)
        achieved = flops / (kms / 1e3) / 1e12
        rng = np.random.default_rng(9)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample * 4, npts), replace=False))
        ref = oracle.oracle_eval_linear_control(p.A, p.x[idx], p.t[idx], p.drift, p.w, tol=1e-26, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval_linear_control(p.A, p.x[idx], p.t[idx], p.drift, p.w,
                                                                             tol=tol, nthreads=nt),
                           p.t, 1 << 18, "same tol, FP64 oracle (one oracle call per point)", one_thread_pts=1 << 10)
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=16 FP64 diagonal path, time-dependent H of linear "
                          "controls; % FP64 vector roofline",
                   value=npts / (ms / 1e3), steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f64",
                   config={"workload": "linear controls dx/ds = diag(m) x + diag(w) beta, beta in [-1,1]^16: "
                                       "diagonal A ~U(0.5,3), m ~U(-1,2) (every fifth 0), w ~U(0.2,2), %d points "
                                       "z~N(0,4I), t~U(0.05,3), FP64, tol %g" % (npts, tol), "npts": npts},
                   roofline={"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                             "frac": achieved / 78.6, "traffic": None,
                             "kernel": "diag_kernel<double, 16, false, false, false, true>",
                             "algorithmic": "sum over points of iterations x 15 n FP64 operations (the "
                                            "per-point weights' exp and expm1 not counted: a lower bound)",
                             "launch_ms": kms},
                   iterations={"mean": float(np.abs(it).mean()), "capped": int(np.sum(it == -2))},
                   accuracy={"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()), "bound": 1e-10},
                   cpu_baseline=cpu)
    elif a.workload == "t5n16":
        npts = a.npts if a.npts != 1 << 16 else 1 << 22
        p = W.workload_paper_norms(16, npts, "linf")
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        tol = a.tol if a.tol is not None else 1e-8
        prob = H.Problem(n=p.n, diagonal=True, hkind="linf", jkind="l1sq", precision="f64", tol=tol, max_iter=20000)
        out = dict(phi=torch.empty(npts, dtype=torch.float64, device=dev),
                   grad=torch.empty(npts, p.n, dtype=torch.float64, device=dev),
                   dphidt=torch.empty(npts, dtype=torch.float64, device=dev),
                   iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
        ms, kms = timed_steps(step, a.steps, a.warmup)
        it = out["iters"].cpu().numpy()
        # per point-iteration: two breakpoint searches (the v-update's and the prox's), each a
        # bitonic sort of m = n rounded up to a power of two (m log m (log m + 1) / 2 min/max
        # operations) and 6 m for the scan and the active sums, plus 15 n for the updates and norms
        m2 = 1 << int(np.ceil(np.log2(p.n)))
        lg = int(np.log2(m2))
        search = m2 * lg * (lg + 1) / 2 + 6.0 * m2
        flops = float(np.sum(np.abs(it)).astype(np.float64) * (2.0 * search + 15.0 * p.n))
        achieved = flops / (kms / 1e3) / 1e12
        rng = np.random.default_rng(10)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample * 4, npts), replace=False))
        ref = oracle.oracle_eval(np.eye(p.n), p.x[idx], p.t[idx], "linf", jkind="l1sq", tol=1e-28, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(np.eye(p.n), p.x[idx], p.t[idx], "linf", jkind="l1sq",
                                                              tol=tol, max_iter=20000, nthreads=nt),
                           p.t, 1 << 20, "same tol, FP64 oracle", one_thread_pts=1 << 10)
        value = npts / (ms / 1e3)
        paper_s = 2.22e-05   # Table 5, n = 16, 16 cores: seconds per evaluation
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=16, J=1/2|y|_1^2, H=|p|_inf, FP64; % FP64 vector roofline",
                   value=value, steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f64",
                   vs_baseline=value * paper_s,
                   config={"workload": "the paper's Table 5 setting: n=16, J = 1/2 |y|_1^2, H = |p|_inf, %d points "
                                       "x~U[-10,10]^16, t~U(0,10], FP64, tol %g" % (npts, tol), "npts": npts},
                   roofline={"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                             "frac": achieved / 78.6, "traffic": None, "kernel": "diag_ext_kernel<double, 16>",
                             "algorithmic": "sum over points of iterations x (2 (m log m (log m + 1) / 2 + 6 m) + "
                                            "15 n) FP64 operations, m = 16 (two sorted breakpoint searches, the "
                                            "updates)",
                             "launch_ms": kms},
                   iterations={"mean": float(np.abs(it).mean()), "capped": int(np.sum(it == -2))},
                   accuracy={"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()), "bound": None,
                             "note": "against the converged oracle (tol 1e-28); the paper's stop rule leaves "
                                     "errors of this size"},
                   paper={"seconds_per_eval": paper_s, "hardware": "16 cores of 2x Xeon E5-2690 (Table 5)",
                          "note": "vs_baseline = value / (1 / seconds_per_eval): another machine, context only"},
                   cpu_baseline=cpu)
    elif a.workload == "pa16":
        npts = a.npts if a.npts != 1 << 16 else 1 << 22
        p = W.workload_paper_a(16, npts)
        HA = p.HA
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        tol = a.tol if a.tol is not None else 1e-8
        prob = H.Problem(np.diag(p.A).copy(), diagonal=True, hkind="al2", HA=HA, precision="f64", tol=tol,
                         max_iter=20000)
        out = dict(phi=torch.empty(npts, dtype=torch.float64, device=dev),
                   grad=torch.empty(npts, p.n, dtype=torch.float64, device=dev),
                   dphidt=torch.empty(npts, dtype=torch.float64, device=dev),
                   iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
        ms, kms = timed_steps(step, a.steps, a.warmup)
        it = out["iters"].cpu().numpy()
        # per point-iteration: the two rotations of the prox (2 n^2 multiply-adds each) and the
        # split-Bregman updates and norms (15 n); the projection's Newton steps not counted
        flops = float(np.sum(np.abs(it)).astype(np.float64) * (4.0 * p.n * p.n + 15.0 * p.n))
        achieved = flops / (kms / 1e3) / 1e12
        rng = np.random.default_rng(9)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample * 4, npts), replace=False))
        ref = oracle.oracle_eval(p.A, p.x[idx], p.t[idx], "al2", HA=HA, tol=1e-28, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(p.A, p.x[idx], p.t[idx], "al2", HA=HA, tol=tol,
                                                              max_iter=20000, nthreads=nt),
                           p.t, 1 << 20, "same tol, FP64 oracle", one_thread_pts=1 << 10)
        value = npts / (ms / 1e3)
        paper_s = 1.04e-05   # Table 4, H = ||.||_A, n = 16: seconds per evaluation on one laptop core
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=16 FP64, H=sqrt(<p,HA p>); % FP64 vector roofline",
                   value=value, steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f64",
                   vs_baseline=value * paper_s,
                   config={"workload": "paper timing-table setting: n=16, D_ii = 1+(i-1)/15, J = 1/2 <y, D^-1 y>, "
                                       "H = sqrt(<p, HA p>), HA = I + 1 1^T, %d points x~U[-10,10]^16, t~U(0,10], "
                                       "FP64, tol %g" % (npts, tol), "npts": npts},
                   roofline={"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                             "frac": achieved / 78.6, "traffic": None,
                             "kernel": "diag_kernel<double, 16, WL2, -, ROT>",
                             "algorithmic": "sum over points of iterations x (4 n^2 + 15 n) FP64 operations (the "
                                            "prox's two rotations, the updates; the projection's Newton steps "
                                            "not counted, so a lower bound)", "launch_ms": kms},
                   iterations={"mean": float(np.abs(it).mean()), "capped": int(np.sum(it == -2))},
                   accuracy={"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()), "bound": None,
                             "note": "against the converged oracle (tol 1e-28); the paper's stop rule leaves "
                                     "errors of this size"},
                   paper={"seconds_per_eval": paper_s, "hardware": "one core of an i5-5300U (Table 4)",
                          "note": "vs_baseline = value / (1 / seconds_per_eval): another machine, context only"},
                   cpu_baseline=cpu)
    elif a.workload in ("c2", "c2wl2"):
        npts = a.npts if a.npts != 1 << 16 else 1 << 20
        hk = "wl1" if a.workload == "c2" else "wl2"
        p = W.round_inputs(W.workload2(npts) if hk == "wl1" else W.workload2_wl2(npts))
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        tol = a.tol if a.tol is not None else 1e-12
        kw = dict(hkind=hk, w=p.w, tol=tol, max_iter=20000, precision="f32")
        out = dict(phi=torch.empty(npts, device=dev), grad=torch.empty(npts, p.n, device=dev),
                   dphidt=torch.empty(npts, device=dev), iters=torch.empty(npts, dtype=torch.int32, device=dev),
                   kstar=torch.empty(npts, dtype=torch.int32, device=dev))

        def step(ev):
            prob = H.Problem(p.A, **kw)
            if ev is not None:
                ev[0].record(stream)
            prob.eval(x, t, out=out)
            if ev is not None:
                ev[1].record(stream)
            del prob
        ms, kms = timed_steps(step, a.steps, a.warmup)
        it = out["iters"].cpu().numpy()
        flops = float(np.sum(np.abs(it)).astype(np.float64) * 2.0 * p.n * p.n)
        achieved = flops / (kms / 1e3) / 1e12
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample * 4, npts), replace=False))
        ref = oracle.oracle_eval(p.A, p.x[idx].astype(np.float64), p.t[idx].astype(np.float64), hk, w=p.w,
                                 tol=1e-28, nthreads=threads)
        g = out["grad"].cpu().numpy()[idx]
        ep = np.linalg.norm(g - ref["grad"], axis=1) / np.maximum(np.linalg.norm(ref["grad"], axis=1), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(p.A, p.x[idx].astype(np.float64),
                                                              p.t[idx].astype(np.float64), hk, w=p.w, tol=tol,
                                                              nthreads=nt),
                           p.t, 1 << 16, "same tol, FP64 oracle", one_thread_pts=64)
        hname = "weighted l1" if hk == "wl1" else "sqrt(<p, diag(w) p>)"
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), n=64 dense FP32%s; %% FP32 MFMA roofline"
                          % ("" if hk == "wl1" else ", H=sqrt(<p,Dp>)"),
                   value=npts / (ms / 1e3), steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f32",
                   config={"workload": "n=64 dense SPD A, H=%s, %d points x~N(0,4I), t~U(0.05,3), FP32, "
                                       "tol %g; step = set-up + evaluation" % (hname, npts, tol), "npts": npts},
                   roofline={"bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                             "frac": achieved / 157.3, "traffic": None, "kernel": "dense_small_kernel<4, 1, 2> (n_pad <= 64)",
                             "algorithmic": "sum over points of iterations x 2 n^2 FLOP", "launch_ms": kms},
                   iterations={"mean": float(np.abs(it).mean()), "capped": int(np.sum(it == -2))},
                   accuracy={"sample": int(len(idx)), "max_rel_err_grad": float(ep.max()), "bound": 1e-6},
                   cpu_baseline=cpu)
    elif a.workload == "c5":  # forward over the union of 4 ellipsoids, then the envelope backward
        npts = a.npts if a.npts != 1 << 16 else 1 << 18
        p = W.round_inputs(W.workload5(npts))
        x = torch.from_numpy(p.x).to(dev)
        t = torch.from_numpy(p.t).to(dev)
        g = torch.from_numpy(np.random.default_rng(5).normal(size=npts).astype(np.float32)).to(dev)
        tol = a.tol if a.tol is not None else 1e-12
        prob = H.Problem(p.A, centres=p.centres, level_set=True, hkind="wl1", w=p.w, precision="f32", tol=tol,
                         max_iter=20000)
        bw_ms = []

        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            out = prob.eval(x, t)
            if ev is not None:
                ev[1].record(stream)
                e2 = torch.cuda.Event(enable_timing=True)
                e2.record(stream)
            b = prob.backward(g, out["grad"], out["dphidt"], out["kstar"])
            if ev is not None:
                e3 = torch.cuda.Event(enable_timing=True)
                e3.record(stream)
                bw_ms.append((e2, e3))
            step.out, step.b = out, b
        for _ in range(a.warmup):
            step(None)
        torch.cuda.synchronize()
        prob.iterations(reset=True)
        ms, kms = timed_steps(step, a.steps, 0)
        passes = prob.iterations(reset=True) / a.steps   # every copy's passes, counted on the device
        bms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in bw_ms]))
        it = step.out["iters"].cpu().numpy()
        flops = float(passes * 2.0 * p.n * p.n)
        achieved = flops / (kms / 1e3) / 1e12
        bw_bytes = npts * (4 * (2 * p.n + 2) + 4 * (p.n + 1) + 4)
        rng = np.random.default_rng(8)
        idx = np.sort(rng.choice(npts, size=min(a.acc_sample, npts), replace=False))
        ref = oracle.oracle_eval(p.A, p.x[idx].astype(np.float64), p.t[idx].astype(np.float64), "wl1", w=p.w,
                                 centres=p.centres, level_set=True, tol=1e-28, nthreads=threads)
        ef = np.abs(step.out["phi"].cpu().numpy()[idx] - ref["phi"]) / np.maximum(np.abs(ref["phi"]), 1)
        cpu = cpu_baseline(lambda idx, nt: oracle.oracle_eval(p.A, p.x[idx].astype(np.float64),
                                                              p.t[idx].astype(np.float64), "wl1", w=p.w,
                                                              centres=p.centres, level_set=True, tol=tol,
                                                              nthreads=nt),
                           p.t, 4096, "forward only, same tol, FP64 oracle", one_thread_pts=8)
        rec.update(metric="Hopf point-evals/sec (φ forward + envelope backward), n=256, union of 4 ellipsoids, FP32",
                   value=npts / (ms / 1e3), steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f32",
                   config={"workload": "n=256, J = min over 4 ellipsoid level sets, H=weighted l1, %d points, FP32, "
                                       "tol %g; step = forward + backward (x, t, A, centres)" % (npts, tol),
                           "npts": npts},
                   roofline={"bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                             "frac": achieved / 157.3, "traffic": measured_traffic_c5(npts, tol),
                             "traffic_unit": "HBM bytes read + written per launch (FETCH_SIZE, WRITE_SIZE scaled)",
                             "kernel": "dense_kernel<2, ...> (FP32 refined)",
                             "algorithmic": "passes of every copy of every point (hopf_problem_iterations) x "
                                            "2 n^2 FLOP", "passes_per_step": passes, "launch_ms": kms},
                   backward={"ms": bms, "hbm_GBps": bw_bytes / (bms / 1e3) / 1e9,
                             "hbm_frac": bw_bytes / (bms / 1e3) / 1e9 / 8000.0,
                             "algorithmic_bytes": bw_bytes},
                   iterations={"mean_attaining_copy": float(np.abs(it).mean()),
                               "mean_per_copy": passes / (npts * p.K)},
                   accuracy={"sample": int(len(idx)), "max_rel_err_phi": float(ef.max()), "bound": 1e-6},
                   cpu_baseline=cpu)
    elif a.workload == "c4":
        # workload 4: 4096 problems, each its own n (log-uniform in [4, 2048]), A, w, t and point
        # count (log-uniform in [1, 4096]), J = min over K = 8 ellipsoid level sets, H = weighted
        # l1, FP32; the whole batch is one call (one persistent launch per kernel class, no host
        # wait between them).  A step creates the problems (host A copied in, FP64 set-up), runs
        # the ragged evaluation and the ragged closest points of the first 64 points of every
        # problem, and releases the problems; each phase is also reported on its own.
        from concurrent.futures import ThreadPoolExecutor
        nall, pall = W.workload4_sizes()
        nprob = len(nall)
        g0 = time.perf_counter()
        def build_A(G, spec):  # the generator's QR and product on the device (FP64 library calls)
            g = torch.from_numpy(G).to(dev)
            q, r = torch.linalg.qr(g)
            sg = torch.sign(torch.diagonal(r))
            q = q * torch.where(sg == 0, torch.ones_like(sg), sg)
            A = (q * torch.from_numpy(spec).to(dev)) @ q.T
            return (0.5 * (A + A.T)).cpu().numpy()
        probs = []
        for i in range(nprob):
            probs.append(W.round_inputs(W.workload4_problem(i, build_A=build_A)))
            if (i + 1) % 512 == 0:
                print("workload 4: %d of %d problems generated (%.0f s)" % (i + 1, nprob, time.perf_counter() - g0),
                      file=sys.stderr, flush=True)

        def tol4(n):  # FP32 increments on exact anchors resolve the step below 1e-6
            return a.tol if a.tol is not None else 1e-12
        specs = [dict(A=p.A, centres=p.centres, level_set=True, hkind="wl1", w=p.w, precision="f32",
                      tol=tol4(p.n), max_iter=20000) for p in probs]
        xs = [torch.from_numpy(p.x).to(dev) for p in probs]
        ts = [torch.from_numpy(p.t).to(dev) for p in probs]
        npts = int(pall.sum())
        # the closest-point leg takes the first CP_PTS points of every problem (a Newton solve per
        # point is several evaluations: the whole batch would take minutes)
        CP_PTS = 64
        ys = [x[:CP_PTS] for x in xs]
        ncp = int(sum(min(int(c), CP_PTS) for c in pall))
        phases = []

        # one step: the problems' FP64 set-up (host A in, batched Gauss-Jordan), the ragged
        # evaluation, the ragged closest points and the release; events split the first three
        def step(ev):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)] if ev is not None else None
            if ev is not None:
                e[0].record(stream)
            hp = H.Problem.batch(specs)
            if ev is not None:
                ev[0].record(stream)
            step.out = H.eval_ragged(hp, xs, ts)
            if ev is not None:
                ev[1].record(stream)
            torch.cuda.synchronize()
            print("workload 4: step evaluated (%.0f s)" % (time.perf_counter() - g0), file=sys.stderr, flush=True)
            step.cp = H.closest_point_ragged(hp, ys, s_tol=1e-7)
            if ev is not None:
                e[1].record(stream)
                phases.append((e[0], ev[0], ev[1], e[1]))
            torch.cuda.synchronize()
            print("workload 4: closest points done (%.0f s)" % (time.perf_counter() - g0), file=sys.stderr, flush=True)
            hp.clear()  # hopf_problem_destroy of every problem
        print("workload 4: evaluating", file=sys.stderr, flush=True)
        ms, kms = timed_steps(step, a.steps, a.warmup)
        print("workload 4: %d steps of %.0f ms" % (a.steps, ms), file=sys.stderr, flush=True)
        setup_ms = float(np.mean([p0.elapsed_time(p1) for p0, p1, _, _ in phases]))
        dist_ms = float(np.mean([p2.elapsed_time(p3) for _, _, p2, p3 in phases]))
        out = step.out
        it = np.abs(out["iters"].cpu().numpy()).astype(np.float64)
        npt = np.repeat(nall, pall).astype(np.float64)
        # counted work: one more evaluation (untimed) with each problem's pass counter read after it
        hp = H.Problem.batch(specs)
        H.eval_ragged(hp, xs, ts)
        passes = np.array([q.iterations(reset=True) for q in hp], np.float64)
        H.closest_point_ragged(hp, ys, s_tol=1e-7)
        passes_d = np.array([q.iterations(reset=True) for q in hp], np.float64)
        del hp
        flops_q = passes * 2.0 * nall.astype(np.float64) ** 2      # per problem, every copy
        flops = float(flops_q.sum())
        flops_d = float((passes_d * 2.0 * nall.astype(np.float64) ** 2).sum())
        # a mixed roofline: per problem max(FLOP / FP32 MFMA peak, bytes / HBM), summed
        off = out["offsets"]
        t_roof = 0.0
        for q in range(nprob):
            bq = float(pall[q] * 4 * (3 * nall[q] + 4) + 4 * nall[q] * nall[q])
            t_roof += max(flops_q[q] / 157.3e12, bq / 8e12)
        achieved = flops / (kms / 1e3) / 1e12
        # accuracy and CPU baseline: one point of each of 48 seeded problems drawn from the whole
        # batch (so the sample has the batch's mix of n); the accuracy reference is the oracle at
        # squared-step tolerance 1e-20 (about 1e-10 relative)
        rng = np.random.default_rng(9)
        qs = np.sort(rng.choice(nprob, size=48, replace=False))
        phi_all = out["phi"].cpu().numpy()
        idxs = {int(q): np.sort(rng.choice(probs[q].npts, size=1, replace=False)) for q in qs}

        def ref_run(q, tol):
            p = probs[q]
            return oracle.oracle_eval(p.A, p.x[idxs[q]].astype(np.float64), p.t[idxs[q]].astype(np.float64),
                                      "wl1", w=p.w, centres=p.centres, level_set=True, tol=tol, nthreads=1)
        c0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda q: ref_run(int(q), tol4(probs[q].n)), qs))
        cpu_s = time.perf_counter() - c0
        cpu_n = sum(len(v) for v in idxs.values())
        with ThreadPoolExecutor(threads) as ex:
            refs = list(ex.map(lambda q: ref_run(int(q), 1e-20), qs))
        errs = []
        for q, ref in zip(qs, refs):
            ph = phi_all[off[q]:off[q + 1]][idxs[int(q)]]
            errs.append(float((np.abs(ph - ref["phi"]) / np.maximum(np.abs(ref["phi"]), 1)).max()))
        rec.update(metric="Hopf point-evals/sec (φ+∇φ), ragged batch of 4096 problems, union of 8 ellipsoids, FP32",
                   value=npts / (ms / 1e3), steps=a.steps, warmup=a.warmup, ms_per_step=ms, dtype="f32",
                   config={"workload": "4096 problems, n = round(logU[4,2048]), A = Q diag(a^2) Q^T (a~U(0.5,3)), "
                                       "w~U(0.5,2), one t~U(0.05,3) per problem, round(logU[1,4096]) points "
                                       "x~N(0,4I), J = min over K=8 ellipsoid level sets (centres ~N(0,9I)), "
                                       "H = weighted l1, FP32, tol 1e-12; step = FP64 set-up of the 4096 "
                                       "problems + ragged evaluation (phi, grad, dphi/dt) of every point + "
                                       "ragged closest points and distances (s_tol 1e-7) of the first %d "
                                       "points of every problem (%d points) + release" % (CP_PTS, ncp),
                           "problems": nprob, "npts": npts, "K": W.W4_K},
                   roofline={"bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                             "frac": achieved / 157.3, "traffic": None,
                             "mixed_frac": t_roof / (kms / 1e3),
                             "mixed": "sum over problems of max(FLOP / 157.3 TFLOP/s, bytes / 8 TB/s), "
                                      "bytes = 4 (3 n + 4) per point + 4 n^2 per problem, over the measured time",
                             "kernel": "dense_small_kernel<...> and dense_kernel<2, ...> (FP32 refined; one "
                                       "launch per class)",
                             "algorithmic": "passes of every copy of every point, counted on the device per problem "
                                            "(hopf_problem_iterations), x 2 n^2 FLOP; the evaluation only",
                             "launch_ms": kms},
                   phases_ms={"setup": setup_ms, "evaluation": kms, "closest_points": dist_ms,
                              "setup_what": "host A copied in + batched FP64 Gauss-Jordan of 4096 problems",
                              "closest_points_tflops": flops_d / (dist_ms / 1e3) / 1e12},
                   iterations={"mean_attaining_copy": float(it.mean()), "max": int(it.max()),
                               "passes_all_copies": float(passes.sum()), "passes_closest_points": float(passes_d.sum())},
                   accuracy={"sample": "1 point of each of %d problems (n %d .. %d)" % (len(qs), nall[qs].min(),
                                                                                    nall[qs].max()),
                             "max_rel_err_phi": max(errs), "bound": 1e-6},
                   cpu_baseline={"value": cpu_n / cpu_s, "unit": "point-evals/s", "cores": threads,
                                 "kind": "oracle", **host_info(),
                                 "sample": "the same %d points (one problem per thread), same tol, FP64 "
                                           "oracle, %d threads (the GPU's CPU share)" % (cpu_n, threads)})
    if a.deterministic:
        rec.setdefault("config", {})["deterministic"] = True
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
