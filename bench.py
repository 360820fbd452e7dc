"""Throughput of the balanced-tree FMM evaluation pass on one MI355X.

One step = fmm_build + fmm_evaluate_tree + fmm_free (tree, lists, P2M, M2M,
M2L, L2L, L2P, P2P) on the 2^20-point Gaussian-mixture cloud (5 levels,
theta 0.5, p 15, FP64), with inputs and outputs resident in HBM.  Prints one
JSON line.  `value` = points per second of the whole step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
    python bench.py --copy-bytes N   (one device-to-device copy of N bytes, for
                                      calibrating the HBM traffic counters)
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

from paper_2002_04894_amd import fmm, workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (and matrix) peak
HBM_PEAK_GBS = 8000.0

# HBM traffic of one M2L launch on the 2^20-point mixture (p 15), from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) of
# `bench.py --steps 1 --warmup 0 --no-cpu --mixed-steps 0 --serve-requests 0
# --tuned-steps 0`, scaled by the same counters on a
# 1 GiB device copy (`bench.py --copy-bytes 1073741824`): FETCH_SIZE read
# 524308 KiB and WRITE_SIZE 1048576 KiB for 1048576 KiB moved each way.
# Valid only for the kernel source it was taken on (hash below).
M2L_COUNTERS = {
    "sources_sha256": "505751c1cb651985704f757fe09a48b2d0e23d888f4d7e6706317efd10ae9ab7",
    "workload": "gmix1m",
    "fetch_kib": 142384087.6875,
    "write_kib": 1016343.9375,
    "fetch_scale": 1048576.0 / 524308.4375,
    "write_scale": 1.0,
}


def m2l_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("m2l_mfma.hip", "tile_layout.h"):
        with open(os.path.join(ROOT, "paper_2002_04894_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def m2l_traffic_gb(workload: str):
    """HBM bytes (GB) per M2L launch from the counters above, or None when
    they were taken on another workload or another version of the kernel."""
    c = M2L_COUNTERS
    if workload != c["workload"] or m2l_sources_sha256() != c["sources_sha256"]:
        return None
    kib = c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]
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
    ap.add_argument("--workload", default="gmix1m")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="steps of the mixed-precision mode timed after the binary64 ones (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests of the served-stream leg run after the timed steps (0: skip)")
    ap.add_argument("--tuned-steps", type=int, default=5,
                    help="steps of the autotuned legs at 1e-6 (mixed allowed, and binary64 only; 0: skip)")
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
    x, y, z, q, w = workloads.workload(args.workload)
    n, L, theta, p = x.shape[0], w["levels"], w["theta"], w["p"]
    dev = lambda a: torch.from_numpy(a).to("cuda")  # noqa: E731
    X, Y, Z, Q = dev(x), dev(y), dev(z), dev(q)
    outs = [torch.empty_like(X) for _ in range(4)]
    stream = torch.cuda.current_stream()

    def step(outs=outs, precision=fmm.FMM_PREC_F64):
        t = fmm.fmm_build(X, Y, Z, L, theta, stream)
        fmm.fmm_evaluate_tree(t, Q, p, *outs, stream, precision=precision)
        return t

    fmm.fmm_set_profiling(True)
    print(f"[bench] {args.workload}: n={n} L={L} theta={theta} p={p}; warm-up", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step().free()
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    phase_sum = {k: 0.0 for k in fmm.PHASES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    last = None
    ev_steps = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for k in range(args.steps):
        tr = step()
        ev_steps[k].record(stream)
        ph = fmm.fmm_last_timings()
        for k in phase_sum:
            phase_sum[k] += ph[k]
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
    ms_step = ms_total / args.steps
    phase_avg = {k: v / args.steps for k, v in phase_sum.items()}

    # dominant kernel: M2L (one launch per step)
    m2l_ms = phase_avg["m2l"]
    m2l_flops = m2l_pairs * m2l_flops_per_pair(p)
    achieved = m2l_flops / (m2l_ms * 1e-3) / 1e12 if m2l_ms > 0 else 0.0
    # orders up to 15 run the matrix-core kernel (binary64 MFMA, whose peak is
    # the binary64 vector peak on this part); higher orders the vector kernel
    mfma_path = p <= 15
    roofline = {
        "kernel": f"k_m2l_mfma<{p}, double>" if mfma_path else "k_m2l",
        "bound": "mfma" if mfma_path else "alu",
        "achieved": round(achieved, 3),
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
        "traffic": m2l_traffic_gb(args.workload),
        "traffic_unit": "GB per launch",
        "launch_ms": round(m2l_ms, 4),
        "pairs": int(m2l_pairs),
        "flops_per_pair": m2l_flops_per_pair(p),
    }
    p2p_ms = phase_avg["p2p"]
    p2p_tflops = p2p_pairs * p2p_flops_per_pair() / (p2p_ms * 1e-3) / 1e12 if p2p_ms > 0 else 0.0

    line = {
        "metric": "points/sec at 1e-6 rel err vs direct sum; served-solve p50/p99 latency",
        "value": round(n / (ms_step * 1e-3), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "step_ms": {"median": round(float(np.median(per_step)), 4), "min": round(per_step[0], 4),
                    "max": round(per_step[-1], 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "levels": L, "theta": theta, "p": p,
                   "generator": w["gen"], "seed": w["seed"]},
        "phase_ms": {k: round(v, 4) for k, v in phase_avg.items()},
        "p2p": {"pairs": int(p2p_pairs), "tflops": round(p2p_tflops, 3),
                "frac_fp64": round(p2p_tflops / FP64_PEAK_TFLOPS, 4)},
        "roofline": roofline,
        "wall_s": round(wall, 3),
    }

    print(f"[bench] {ms_step:.1f} ms per step", file=sys.stderr, flush=True)
    mouts = None
    if args.mixed_steps > 0:
        mouts = [torch.empty_like(X) for _ in range(4)]
        line["mixed"] = mixed_leg(step, mouts, outs, n, args.mixed_steps, stream, torch)

    line["accuracy"] = gpu_direct_gate(X, Y, Z, Q, outs, torch)
    if mouts is not None:
        line["mixed"]["accuracy"] = gpu_direct_gate(X, Y, Z, Q, mouts, torch)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
    if args.tuned_steps > 0 and n <= TUNED_MAX_N:
        line["tuned"] = tuned_legs(X, Y, Z, Q, L, args.tuned_steps, stream, torch)
    if args.serve_requests > 0:
        line["serving"] = serving_leg(args.serve_requests)
    print(json.dumps(line), flush=True)


TUNED_MAX_N = 1 << 22  # the tuned legs calibrate on clouds of the workload's size


def tuned_legs(X, Y, Z, Q, L, steps, stream, torch, tol: float = 1e-6) -> dict:
    """The workload at the metric's accuracy with theta, p and precision
    picked by the autotuner (serve.Tuner, calibrated on the GPU at this level
    count, theta 0.4, 0.5 and 0.6, orders 1..15): its choice with mixed
    precision allowed, and its choice with every candidate in binary64.
    Each: ms per step (build + evaluate) and the error against the direct sum
    at 10,000 sampled points (gpu_direct_gate)."""
    from paper_2002_04894_amd import serve
    n = X.numel()
    tuner = serve.Tuner()
    t0 = time.perf_counter()
    tuner.calibrate(levels=(L,), thetas=(0.4, 0.5, 0.6), orders=range(1, 16))
    cal_s = time.perf_counter() - t0
    out = {"tol": tol, "calibration_s": round(cal_s, 2)}
    legs = {"mixed_allowed": tuner.choose(n, tol), "f64": tuner.choose(n, tol, allow_mixed=False)}
    for name, (lv, t_, p_, pr) in legs.items():
        o = [torch.empty_like(X) for _ in range(4)]

        def step():
            tr = fmm.fmm_build(X, Y, Z, lv, t_, stream)
            fmm.fmm_evaluate_tree(tr, Q, p_, *o, stream, precision=pr)
            return tr

        step().free()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        last = None
        for _ in range(steps):
            tr = step()
            if last is not None:
                last.free()
            last = tr
        ev1.record(stream)
        torch.cuda.synchronize()
        last.free()
        ms = ev0.elapsed_time(ev1) / steps
        out[name] = {"levels": lv, "theta": t_, "p": p_, "precision": "mixed" if pr else "f64",
                     "ms_per_step": round(ms, 4), "value": round(n / (ms * 1e-3), 1), "unit": "points/s",
                     "accuracy": gpu_direct_gate(X, Y, Z, Q, o, torch)}
    return out


def serving_leg(nreq: int) -> dict:
    """The served-solve latency half of the metric: a stream of `nreq`
    requests (Poisson arrivals at 200/s, N log-uniform in [1e3, 2e5], three
    distributions, accuracy 1e-4 or 1e-8) through the continuous-batching
    server with 6 workers, after calibrating its tuner."""
    from paper_2002_04894_amd import serve
    r = serve.run_stream(nreq, 200.0, 6, check_every=max(1, nreq // 2))
    keep = ("requests", "failed", "p50_ms", "p99_ms", "mean_ms", "requests_per_s", "points_per_s", "choices",
            "accuracy_ok")
    out = {k: r[k] for k in keep}
    out["rate_per_s"] = 200.0
    out["workers"] = 6
    return out


def gpu_direct_gate(X, Y, Z, Q, outs, torch, k: int = 10_000) -> dict:
    """Relative error vs the direct sum (eq. 2.1) at k sampled points,
    computed on the GPU: a 2-level tree with theta = 0 makes every pair of
    leaves strongly connected, so the evaluation at the sampled points, given
    as separate targets, is the plain pairwise sum (no expansions; a target's
    own source is skipped).  That path is the P2P that the parity tests check
    against the oracle."""
    n = X.numel()
    tg = workloads.sample_targets(n, k, seed=1)
    idx = torch.from_numpy(tg).to("cuda")
    T = [a.index_select(0, idx).contiguous() for a in (X, Y, Z)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = fmm.fmm_build_ex(X, Y, Z, 2, 0.0, targets=tuple(T))
    d = [torch.empty(k, dtype=torch.float64, device="cuda") for _ in range(4)]
    fmm.fmm_evaluate_targets(tree, Q, 0, *d)
    torch.cuda.synchronize()
    direct_ms = 1e3 * (time.perf_counter() - t0)
    tree.free()
    d = [a.cpu().numpy() for a in d]
    g = [o.index_select(0, idx).cpu().numpy() for o in outs]
    ephi = float(np.linalg.norm(g[0] - d[0]) / np.linalg.norm(d[0]))
    eE = float(np.linalg.norm(np.concatenate(g[1:]) - np.concatenate(d[1:])) / np.linalg.norm(np.concatenate(d[1:])))
    return {"targets": k, "method": "GPU direct sum at sampled targets (theta = 0, all P2P)", "rel_err_phi": ephi,
            "rel_err_E": eE, "ok": bool(ephi <= 1e-6 and eE <= 1e-6), "direct_sum_ms": round(direct_ms, 3)}


def mixed_leg(step, mouts, outs, n, steps, stream, torch):
    """The same step in mixed precision (binary32 M2L, the rest binary64):
    one warm-up and `steps` timed steps, its M2L time, and its difference to
    the binary64 result just computed (normwise, potential and field)."""
    step(mouts, fmm.FMM_PREC_MIXED).free()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    m2l = 0.0
    e0.record(stream)
    last = None
    for _ in range(steps):
        tr = step(mouts, fmm.FMM_PREC_MIXED)
        m2l += fmm.fmm_last_timings()["m2l"]
        if last is not None:
            last.free()
        last = tr
    e1.record(stream)
    torch.cuda.synchronize()
    last.free()
    ms = e0.elapsed_time(e1) / steps
    dphi = float(torch.linalg.norm(mouts[0] - outs[0]) / torch.linalg.norm(outs[0]))
    dE = float(torch.sqrt(sum(torch.sum((a - b) ** 2) for a, b in zip(mouts[1:], outs[1:])))
               / torch.sqrt(sum(torch.sum(b ** 2) for b in outs[1:])))
    return {"dtype": "f32 m2l, f64 rest", "steps": steps, "ms_per_step": round(ms, 4),
            "value": round(n / (ms * 1e-3), 1), "unit": "points/s", "m2l_ms": round(m2l / steps, 4),
            "rel_diff_vs_f64": {"phi": dphi, "E": dE}}


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


def cpu_baseline(w):
    """The CPU oracle (single thread, as it stands) on a bounded sample of the
    same workload: the same generator, theta and p with 16,384 points and 3
    levels (the same 32 points per leaf), the full tree and upward pass, and
    the evaluation at every point of every 8th leaf (64 of 512 leaves)."""
    import oracle
    ns, Ls = 16_384, 3
    x, y, z, q, _ = workloads.workload("gmix1m", n=ns)
    leaves = np.arange(0, 8 ** Ls, 8)
    t0 = time.perf_counter()
    tr = oracle.Tree(x, y, z, Ls, w["theta"])
    tr.evaluate(q, w["p"], leaves=leaves)
    dt = time.perf_counter() - t0
    s = tr.start(Ls)
    pts = int(sum(s[b + 1] - s[b] for b in leaves))
    return {"value": round(pts / dt, 2), "unit": "points/s", "cores": 1, "kind": "oracle",
            "seconds": round(dt, 2),
            "sample": f"gmix generator, n={ns}, levels={Ls}, theta={w['theta']}, p={w['p']}; full tree + upward "
                      f"pass, evaluation at the {pts} points of {len(leaves)} of {8 ** Ls} leaves"}


if __name__ == "__main__":
    main()
