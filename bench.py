"""Throughput of the balanced-tree FMM evaluation pass on one MI355X.

One step = fmm_build + fmm_evaluate_tree + fmm_free (tree, lists, P2M, M2M,
M2L, L2L, L2P, P2P), with inputs and outputs resident in HBM.  The default
workload is the largest one-GPU configuration: 2^27 Plummer points (scale
radius 0.02, charges in [-1, 1]), 7 levels, with theta, p and the precision
autotuned to 1e-6 against the direct sum at 10,000 sampled points (the
autotuning time is reported apart, outside the timed steps).  Beside it: the
binary64 leg at its own tuned setting, the oracle on the host cores, and the
served stream of 4,000 requests (p50/p99 latency).  Prints one JSON line;
`value` = points per second of the whole step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--fixed] [--no-cpu]
    python bench.py --copy-bytes N   (one device-to-device copy of N bytes, for
                                      calibrating the HBM traffic counters)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2002_04894_amd import fmm, workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6        # MI355X binary64 vector (and matrix) peak
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X binary32 matrix peak (dense)
LANE_M2L_MAX_P = 14            # mixed precision: the per-lane M2L kernel up to this order, 16x16 tiles above


def quad_m2l(p: int) -> bool:
    """binary64 M2L runs four lanes per pair at these orders (16x16 tiles at
    14 and 15)"""
    return p <= 13 or 16 <= p <= 20
HBM_PEAK_GBS = 8000.0

# HBM traffic of one M2L launch, per kernel and workload: from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of the bench
# command named in the summary under profiles/, scaled by the same counters
# on a 1 GiB device copy (`bench.py --copy-bytes 1073741824`; FETCH_SIZE read
# 524308 KiB and WRITE_SIZE 1048576 KiB for 1048576 KiB moved each way).  An
# entry holds only for the kernel source it was taken on (hash), else None.
COPY_FETCH_SCALE = 1048576.0 / 524308.4375
COPY_WRITE_SCALE = 1.0
M2L_COUNTERS: dict = {  # (kernel, n, theta) -> {"sources_sha256", "fetch_kib", "write_kib"}
    # profiles/m2l_counters_plummer134m.md (theta 0.6, p 12): mixed precision and binary64
    ("k_m2l_lane<12>", 1 << 27, 0.6): {
        "sources_sha256": "1e390d48b53daa9cf247241abb1bb3e2ea4ac8e19a66424d12fd0d64fb5aefd5",
        "fetch_kib": 3976133030.875,
        "write_kib": 479565723.84375,
    },
    ("k_m2l_quad<12>", 1 << 27, 0.6): {
        "sources_sha256": "7506a256e0c87c880341bd40c953d8f76270fd36dfee7dc9c089359c5c6d4cc4",
        "fetch_kib": 10978627894.625,
        "write_kib": 20261523.8125,
    },
    # the binary64 leg's tuned setting (theta 0.55, p 10)
    ("k_m2l_quad<10>", 1 << 27, 0.55): {
        "sources_sha256": "7506a256e0c87c880341bd40c953d8f76270fd36dfee7dc9c089359c5c6d4cc4",
        "fetch_kib": 8859291027.4375,
        "write_kib": 6013182.5,
    },
}


def m2l_sources_sha256(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    files = {"k_m2l_lane": ("m2l_lane.hip", "lane_ops.h"), "k_m2l_quad": ("m2l_quad.hip", "lane_ops.h")}.get(
        kernel.split("<")[0], ("m2l_mfma.hip",))
    for f in files + ("tile_layout.h",):
        with open(os.path.join(ROOT, "paper_2002_04894_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def m2l_traffic_gb(kernel: str, n: int, theta: float):
    """HBM bytes (GB) per M2L launch from the counters above, or None when
    none were taken for this kernel, workload and kernel source."""
    c = M2L_COUNTERS.get((kernel, n, theta))
    if c is None or m2l_sources_sha256(kernel) != c["sources_sha256"]:
        return None
    kib = c["fetch_kib"] * COPY_FETCH_SCALE + c["write_kib"] * COPY_WRITE_SCALE
    return round(kib * 1024 / 1e9, 2)


def m2l_flops_per_pair(p: int) -> int:
    """Algorithmic flops of one rotational M2L (Section 2.1.3): two rotations
    with dense per-degree blocks, sum_n (2n+1)^2 multiply-adds each, plus the
    z-axis translation, sum_m (p+1-|m|)^2 multiply-adds; 2 flops each."""
    rot = sum((2 * n + 1) ** 2 for n in range(p + 1))
    zt = sum((p + 1 - abs(m)) ** 2 for m in range(-p, p + 1))
    return 2 * (2 * rot + zt)


def p2p_flops_per_pair() -> int:
    """Near-field interaction: 3 sub, 5 for r^2, 1 rsqrt, 9 for phi and E."""
    return 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plummer134m")
    ap.add_argument("--fixed", action="store_true",
                    help="time the workload's fixed theta and p in binary64 instead of the autotuned setting")
    ap.add_argument("--tol", type=float, default=1e-6, help="accuracy the autotuner must reach")
    ap.add_argument("--setting", default="",
                    help="THETA,P,PRECISION (f64 or mixed): time this setting, skipping the autotuner "
                         "(for profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--f64-steps", type=int, default=3,
                    help="steps of the binary64 leg beside the autotuned (mixed) one (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=4000,
                    help="requests of the served-stream leg run after the timed steps (0: skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run one plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_bytes:
        copy_probe(args.copy_bytes)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_gen = time.perf_counter()
    x, y, z, q, w = workloads.workload(args.workload)
    n, L = x.shape[0], w["levels"]
    dev = lambda a: torch.from_numpy(a).to("cuda")  # noqa: E731
    X, Y, Z, Q = dev(x), dev(y), dev(z), dev(q)
    del x, y, z, q
    torch.cuda.synchronize()
    log(f"{args.workload}: n={n} L={L}; inputs on the device after {time.perf_counter() - t_gen:.1f} s")
    stream = torch.cuda.current_stream()
    fmm.fmm_set_profiling(True)

    if args.fixed:
        tune = {"theta": w["theta"], "p": w["p"], "precision": fmm.FMM_PREC_F64}
        tuned_info = None
    elif args.setting:
        th_s, p_s, pr_s = args.setting.split(",")
        tune = {"theta": float(th_s), "p": int(p_s),
                "precision": fmm.FMM_PREC_MIXED if pr_s == "mixed" else fmm.FMM_PREC_F64}
        tuned_info = None
    else:
        tune, tuned_info = autotune(X, Y, Z, Q, L, args.tol, stream, torch, f64=args.f64_steps > 0)
    theta, p, prec = tune["theta"], tune["p"], tune["precision"]
    outs = [torch.empty_like(X) for _ in range(4)]
    leg = timed_leg(X, Y, Z, Q, L, theta, p, prec, outs, args.steps, args.warmup, stream, torch)
    ms_step = leg["ms_per_step"]
    mixed_path = prec == fmm.FMM_PREC_MIXED and p <= 15
    line = {
        "metric": "points/sec at 1e-6 rel err vs direct sum; served-solve p50/p99 latency",
        "value": round(n / (ms_step * 1e-3), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "step_ms": leg["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (binary32 M2L, binary64 rest)" if mixed_path else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "levels": L, "theta": theta, "p": p,
                   "precision": "mixed" if mixed_path else "f64", "generator": w["gen"], "seed": w["seed"],
                   "tuned": tuned_info is not None},
        "phase_ms": leg["phase_ms"],
        "p2p": leg["p2p"],
        "roofline": leg["roofline"],
        "wall_s": leg["wall_s"],
    }
    log(f"{ms_step:.1f} ms per step")
    line["accuracy"] = gpu_direct_gate(X, Y, Z, Q, outs, torch)
    if tuned_info is not None:
        line["autotune"] = tuned_info
    if args.f64_steps > 0 and prec != fmm.FMM_PREC_F64 and tuned_info is not None:
        f = tuned_info["f64_choice"]
        fouts = [torch.empty_like(X) for _ in range(4)]
        fl = timed_leg(X, Y, Z, Q, L, f["theta"], f["p"], fmm.FMM_PREC_F64, fouts, args.f64_steps, 1, stream,
                       torch)
        dphi, dE = rel_diff(outs, fouts, torch)
        line["f64"] = {"theta": f["theta"], "p": f["p"], "steps": args.f64_steps,
                       "ms_per_step": round(fl["ms_per_step"], 4), "value": round(n / (fl["ms_per_step"] * 1e-3), 1),
                       "unit": "points/s", "phase_ms": fl["phase_ms"], "roofline": fl["roofline"],
                       "accuracy": gpu_direct_gate(X, Y, Z, Q, fouts, torch),
                       "rel_diff_headline_vs_f64": {"phi": dphi, "E": dE}}
        line["mixed_over_f64"] = round(fl["ms_per_step"] / ms_step, 3)
        del fouts
    del outs
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, theta, p)
    if args.serve_requests > 0:
        line["serving"] = serving_leg(args.serve_requests)
    print(json.dumps(line), flush=True)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_leg(X, Y, Z, Q, L, theta, p, prec, outs, steps, warmup, stream, torch) -> dict:
    """`warmup` untimed steps, then `steps` timed ones, each fmm_build +
    fmm_evaluate_tree (+ the previous step's fmm_free), bracketed by
    synchronisations; per-phase times from the library's HIP events on the
    call stream; the M2L roofline line of the dominant kernel."""
    n = X.numel()

    def step():
        t = fmm.fmm_build(X, Y, Z, L, theta, stream)
        fmm.fmm_evaluate_tree(t, Q, p, *outs, stream, precision=prec)
        return t

    for _ in range(warmup):
        step().free()
    torch.cuda.synchronize()
    log(f"timing {steps} steps: theta={theta} p={p} precision={'mixed' if prec else 'f64'}")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    phase_sum = {k: 0.0 for k in fmm.PHASES}
    ev_steps = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    ev0.record(stream)
    last = None
    for k in range(steps):
        tr = step()
        ev_steps[k].record(stream)
        ph = fmm.fmm_last_timings()
        for key in phase_sum:
            phase_sum[key] += ph[key]
        if last is not None:
            last.free()
        last = tr
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    per_step = sorted(a.elapsed_time(b) for a, b in zip([ev0] + ev_steps[:-1], ev_steps))
    m2l_pairs, p2p_pairs = fmm.fmm_tree_stats(last)
    last.free()
    ms_step = ms_total / steps
    phase_avg = {k: v / steps for k, v in phase_sum.items()}
    m2l_ms = phase_avg["m2l"]
    achieved = m2l_pairs * m2l_flops_per_pair(p) / (m2l_ms * 1e-3) / 1e12 if m2l_ms > 0 else 0.0
    mixed = prec == fmm.FMM_PREC_MIXED and p <= 15
    if mixed and p <= LANE_M2L_MAX_P:
        kernel, bound, peak = f"k_m2l_lane<{p}>", "mfma", FP32_MFMA_PEAK_TFLOPS
    elif not mixed and quad_m2l(p):
        kernel, bound, peak = f"k_m2l_quad<{p}>", "mfma", FP64_PEAK_TFLOPS
    else:
        kernel = f"k_m2l_mfma<{p}, {'float' if mixed else 'double'}>"
        bound, peak = "mfma", FP32_MFMA_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
    roofline = {
        "kernel": kernel, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4), "traffic": m2l_traffic_gb(kernel, n, theta),
        "traffic_unit": "GB per launch", "launch_ms": round(m2l_ms, 4), "pairs": int(m2l_pairs),
        "flops_per_pair": m2l_flops_per_pair(p),
    }
    p2p_ms = phase_avg["p2p"]
    p2p_tflops = p2p_pairs * p2p_flops_per_pair() / (p2p_ms * 1e-3) / 1e12 if p2p_ms > 0 else 0.0
    return {"ms_per_step": ms_step,
            "step_ms": {"median": round(float(np.median(per_step)), 4), "min": round(per_step[0], 4),
                        "max": round(per_step[-1], 4)},
            "phase_ms": {k: round(v, 4) for k, v in phase_avg.items()},
            "p2p": {"pairs": int(p2p_pairs), "tflops": round(p2p_tflops, 3),
                    "frac_fp64": round(p2p_tflops / FP64_PEAK_TFLOPS, 4)},
            "roofline": roofline, "wall_s": round(wall, 3)}


def rel_diff(a, b, torch):
    dphi = float(torch.linalg.norm(a[0] - b[0]) / torch.linalg.norm(b[0]))
    dE = float(torch.sqrt(sum(torch.sum((u - v) ** 2) for u, v in zip(a[1:], b[1:])))
               / torch.sqrt(sum(torch.sum(v ** 2) for v in b[1:])))
    return dphi, dE


def autotune(X, Y, Z, Q, L, tol, stream, torch, thetas=(0.5, 0.55, 0.6, 0.65, 0.7),
             f64: bool = True) -> tuple[dict, dict]:
    """theta and p (and the precision) for accuracy `tol` on this workload,
    chosen by measurement (Section 3.2: the response to the parameters is
    convex, so a small search finds the optimum):
      1. a proxy of the workload -- every 64th point, 2 levels fewer (the
         same points per leaf) -- gives the error of every (theta, p) against
         its direct sum at 10,000 points, in mixed precision;
      2. per theta the smallest order whose proxy error is within tol / 2,
         timed for one step on the workload itself;
      3. the fastest of these whose error on the workload, against the direct
         sum at 10,000 sampled points, is within tol wins; a candidate that
         misses tol is retried one order higher.
    The binary64 leg beside it (f64) is tuned the same way over the thetas
    that had a mixed candidate (binary64 proxy errors, one timed step each),
    the fastest within tol winning.  Returns (choice, report)."""
    t0 = time.perf_counter()
    n = X.numel()
    k = 64
    Lp = max(1, L - 2)
    sub = torch.arange(0, n, k, device="cuda")
    Xs, Ys, Zs, Qs = (a.index_select(0, sub).contiguous() for a in (X, Y, Z, Q))
    ns = Xs.numel()
    tg = workloads.sample_targets(ns, min(10_000, ns), seed=3)
    tgi = torch.from_numpy(tg).to("cuda")
    ref = direct_at(Xs, Ys, Zs, Qs, tgi, torch)
    orders = range(4, 16)
    proxy = {}
    o = [torch.empty_like(Xs) for _ in range(4)]

    def probe(th, precs):
        tr = fmm.fmm_build(Xs, Ys, Zs, Lp, th, stream)
        for p in orders:
            for prec in precs:
                fmm.fmm_evaluate_tree(tr, Qs, p, *o, stream, precision=prec)
                g = [a.index_select(0, tgi).cpu().numpy() for a in o]
                proxy[(th, p, prec)] = max(rel_err(g, ref))
        tr.free()

    for th in thetas:
        probe(th, (fmm.FMM_PREC_MIXED,))
    cal_proxy_s = time.perf_counter() - t0
    log(f"autotune: proxy of {ns} points at {Lp} levels, {len(proxy)} settings in {cal_proxy_s:.1f} s")

    outs = [torch.empty_like(X) for _ in range(4)]
    tried = []

    def first_order(th, prec):
        for p in orders:
            if proxy.get((th, p, prec), math.inf) <= tol / 2:
                return p
        return None

    def run(th, p, prec):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tr = fmm.fmm_build(X, Y, Z, L, th, stream)
        fmm.fmm_evaluate_tree(tr, Q, p, *outs, stream, precision=prec)
        tr.free()
        e1.record(stream)
        torch.cuda.synchronize()
        acc = gpu_direct_gate(X, Y, Z, Q, outs, torch)
        err = max(acc["rel_err_phi"], acc["rel_err_E"])
        rec = {"theta": th, "p": p, "precision": "mixed" if prec else "f64", "ms": round(e0.elapsed_time(e1), 2),
               "err": err, "proxy_err": proxy.get((th, p, prec))}
        tried.append(rec)
        log(f"autotune: theta={th} p={p} {rec['precision']}: {rec['ms']:.0f} ms, error {err:.2e}")
        return rec

    # mixed precision: per theta the smallest order whose proxy error is
    # within tol / 2, one timed step each on the workload; the fastest that
    # meets tol on it wins
    best = None
    for th in thetas:
        p = first_order(th, fmm.FMM_PREC_MIXED)
        if p is None:
            continue
        pr = fmm.FMM_PREC_MIXED
        for _ in range(2):
            rec = run(th, p, pr)
            if rec["err"] <= tol:
                if best is None or rec["ms"] < best["ms"]:
                    best = rec
                break
            p += 1
            if p > 15:
                break
    if best is None:
        raise RuntimeError(f"no setting reached {tol} on this workload")
    # binary64: the same search over the thetas that had a mixed candidate
    # (M2L costs more per pair in binary64, so its best theta can be smaller)
    best64 = None
    for th in sorted({r["theta"] for r in tried}) if f64 else ():
        probe(th, (fmm.FMM_PREC_F64,))
        p = first_order(th, fmm.FMM_PREC_F64)
        if p is None:
            continue
        rec = run(th, p, fmm.FMM_PREC_F64)
        if rec["err"] <= tol and (best64 is None or rec["ms"] < best64["ms"]):
            best64 = rec
    if best64 is None:  # none met tol on the workload: the mixed winner's theta, its binary64 order
        best64 = {"theta": best["theta"], "p": first_order(best["theta"], fmm.FMM_PREC_F64) or 15}
    report = {"tol": tol, "proxy": {"points": ns, "levels": Lp, "settings": len(proxy), "seconds": round(cal_proxy_s, 2)},
              "tried": tried, "seconds": round(time.perf_counter() - t0, 2),
              "f64_choice": {"theta": best64["theta"], "p": best64["p"]}}
    choice = {"theta": best["theta"], "p": best["p"],
              "precision": fmm.FMM_PREC_MIXED if best["precision"] == "mixed" else fmm.FMM_PREC_F64}
    return choice, report


def direct_at(X, Y, Z, Q, idx, torch):
    """Direct sum (eq. 2.1) at the points idx, on the GPU: a 2-level tree
    with theta = 0 makes every pair of leaves strongly connected, so the
    evaluation at those points, given as separate targets, is the plain
    pairwise sum (a target's own source is skipped)."""
    T = [a.index_select(0, idx).contiguous() for a in (X, Y, Z)]
    tree = fmm.fmm_build_ex(X, Y, Z, 2, 0.0, targets=tuple(T))
    d = [torch.empty(idx.numel(), dtype=torch.float64, device="cuda") for _ in range(4)]
    fmm.fmm_evaluate_targets(tree, Q, 0, *d)
    torch.cuda.synchronize()
    tree.free()
    return [a.cpu().numpy() for a in d]


def rel_err(g, d):
    ephi = float(np.linalg.norm(g[0] - d[0]) / np.linalg.norm(d[0]))
    eE = float(np.linalg.norm(np.concatenate(g[1:]) - np.concatenate(d[1:])) / np.linalg.norm(np.concatenate(d[1:])))
    return ephi, eE


def serving_leg(nreq: int) -> dict:
    """The served-solve latency half of the metric: a stream of `nreq`
    requests (Poisson arrivals at 200/s, N log-uniform in [1e3, 2e5], three
    distributions, accuracy 1e-4 or 1e-8) through the continuous-batching
    server with 6 workers, after calibrating its tuner."""
    from paper_2002_04894_amd import serve
    r = serve.run_stream(nreq, 200.0, 6, check_every=max(1, nreq // 8))
    keep = ("requests", "failed", "p50_ms", "p99_ms", "mean_ms", "requests_per_s", "points_per_s", "choices",
            "accuracy_ok", "device_overlap", "peak_concurrency", "deferred", "exact_over_estimate_max",
            "calibration_s")
    out = {k: r[k] for k in keep}
    out["rate_per_s"] = 200.0
    out["workers"] = 6
    return out


def gpu_direct_gate(X, Y, Z, Q, outs, torch, k: int = 10_000) -> dict:
    """Relative error vs the direct sum (eq. 2.1) at k sampled points
    (direct_at: the P2P path that the parity tests check against the oracle)."""
    n = X.numel()
    tg = workloads.sample_targets(n, k, seed=1)
    idx = torch.from_numpy(tg).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = direct_at(X, Y, Z, Q, idx, torch)
    direct_ms = 1e3 * (time.perf_counter() - t0)
    g = [o.index_select(0, idx).cpu().numpy() for o in outs]
    ephi, eE = rel_err(g, d)
    return {"targets": k, "method": "GPU direct sum at sampled targets (theta = 0, all P2P)", "rel_err_phi": ephi,
            "rel_err_E": eE, "ok": bool(ephi <= 1e-6 and eE <= 1e-6), "direct_sum_ms": round(direct_ms, 3)}


def copy_probe(nbytes: int):
    """One device-to-device copy of `nbytes` (after one untimed warm-up copy),
    whose FETCH_SIZE / WRITE_SIZE counters calibrate the traffic figures."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 8}), flush=True)


def cpu_baseline(w, theta: float, p: int, ns: int = 1 << 18) -> dict:
    """The CPU oracle as it stands (binary64, the paper's rotational M2L,
    OpenMP threads over boxes and leaves on every host core) timed on a
    bounded sample of the same workload: the same generator with `ns` points
    at the level count that keeps the workload's points per leaf, at the
    benchmarked theta and p; tree, lists and the evaluation at every point
    (the whole step).  points/s = ns / seconds."""
    import math

    import oracle
    per_leaf = w["n"] / 8 ** w["levels"]
    Ls = max(0, round(math.log(ns / per_leaf, 8)))
    x, y, z, q, _ = workloads.workload(w_name(w), n=ns)
    # the host cores this process may use (the box's share when OMP_NUM_THREADS says so)
    cores = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0)))
    oracle.set_m2l_form(True)
    t0 = time.perf_counter()
    tr = oracle.Tree(x, y, z, Ls, theta)
    tr.evaluate(q, p)
    dt = time.perf_counter() - t0
    oracle.set_m2l_form(False)
    return {"value": round(ns / dt, 2), "unit": "points/s", "cores": cores, "kind": "oracle",
            "seconds": round(dt, 2),
            "sample": f"{w['gen']} generator as in the workload, n={ns}, levels={Ls} ({ns / 8 ** Ls:.0f} points "
                      f"per leaf), theta={theta}, p={p}; tree + lists + evaluation at all points, rotational M2L, "
                      f"{cores} threads"}


def w_name(w) -> str:
    return next(k for k, v in workloads.WORKLOADS.items() if v["gen"] == w["gen"] and v.get("a") == w.get("a")
                and v["levels"] == w["levels"] and v["n"] == w["n"])


if __name__ == "__main__":
    main()
