#!/usr/bin/env python3
"""Throughput of one full step of the non-metric Vicsek model on one MI355X.

Workload (synthetic, seeded): N = 2^20 particles uniform in a periodic box of
side L = 2^20, headings uniform, k = 7 topological neighbours, v0 = 64,
eta = 0.2, Philox seed 0; beside the k-NN list the metric cutoff list is
rebuilt every step with r_c^2 = 2,336,407 (a mean of 7 neighbours).

One timed step = every stage of the hot path on the GPU:
  nm_bin_step      cell binning (histogram, scan, scatter + noise + unit vectors)
  nm_knn_align     k-NN lists fused with Eq. (2) alignment and Eq. (1) move
  nm_metric_list   metric cutoff list (count, scan, fill; capacity preset)
Inputs are resident in HBM before timing starts.  The value is particle-steps
per second (N * steps / wall time of the timed steps).

The dominant kernel (the fused k-NN + alignment kernel) is bracketed by HIP
events on the stream it runs on; its roofline entry prices the step's
compulsory traffic, 24 + 4k bytes per particle-step (read x, y, theta; write
the k indices and x', y', theta'), against the 8 TB/s HBM peak.

cpu_baseline: the brute-force oracle timed on the host on a sample of the same
workload (a few thousand query particles of the N = 2^20 system, all stages).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s (k=7 kNN rebuild + align) at N=1M; batched p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--k", type=int, default=7)
    ap.add_argument("--cell-w", type=int, default=0, help="cell width (0: built-in choice)")
    ap.add_argument("--no-metric", action="store_true", help="time the k-NN step only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def cpu_baseline(x, y, th, k, rc2, box, target_s):
    """Oracle (brute force, all host threads) on sampled query rows of the same system."""
    import numpy as np

    import oracle
    from paper_2103_10239_amd import workloads

    n = len(x)
    rng = np.random.default_rng(11)

    def run(rows):
        t0 = time.perf_counter()
        nbr, _ = oracle.knn(x, y, box, k, rows=rows, with_d2=False)
        oracle.align_step(x, y, th, box, nbr=nbr, v0=64, eta=0.2, seed=workloads.NOISE_SEED, rows=rows)
        if rc2 is not None:
            oracle.metric_list(x, y, box, rc2, rows=rows, with_d2=False)
        return time.perf_counter() - t0

    probe = rng.choice(n, size=min(256, n), replace=False).astype(np.int32)
    t_probe = max(run(probe), 1e-6)
    m = int(min(n, max(256, len(probe) * target_s / t_probe)))
    rows = rng.choice(n, size=m, replace=False).astype(np.int32)
    t = run(rows)
    return {"value": m / t, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{m} sampled particles of the N={n} system: brute-force k-NN rows, "
                      f"Eq. 1-2 step{' and metric rows' if rc2 is not None else ''}; {t:.1f} s",
            "seconds": t}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path has no "
              "multi-GPU mode in this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_10239_amd as nm
    from paper_2103_10239_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, k, box = args.n, args.k, workloads.BOX
    rc2 = None if args.no_metric else workloads.rc2_for_mean(n, 7.0)
    cell_w = args.cell_w or nm.suggest_cell_w(n, box, 4.0)

    x, y, th = workloads.uniform(n)
    p = nm.make_params(box, v0=64, eta=0.2, include_self=1, seed=workloads.NOISE_SEED)
    ws = nm.Workspace(n, box, cell_w, dev)
    X = torch.as_tensor(x).to(dev)
    Y = torch.as_tensor(y).to(dev)
    T = torch.as_tensor(th).to(dev)
    Xb, Yb, Tb = torch.empty_like(X), torch.empty_like(Y), torch.empty_like(T)
    nbr = torch.empty((n, k), dtype=torch.int32, device=dev)
    offsets = torch.empty(n + 1, dtype=torch.int32, device=dev)
    idx = None
    if rc2 is not None:
        # From the disordered start the aligned groups cluster, and the mean metric
        # degree climbs steadily (7 at step 0, about 31 by step 375), so the index
        # array gets a fixed capacity of 160 per particle; an overflow would be
        # reported by nm_check and fail the run.
        idx = torch.empty(160 * n, dtype=torch.int32, device=dev)

    state = {"x": X, "y": Y, "t": T, "xb": Xb, "yb": Yb, "tb": Tb, "step": 0}

    def one_step(ev=None):
        s = state
        nm.bin_step(ws, s["x"], s["y"], s["t"], p, s["step"])
        if ev is not None:
            ev[0].record()
        nm.knn_align(ws, k, p, s["t"], nbr, s["xb"], s["yb"], s["tb"])
        if ev is not None:
            ev[1].record()
        if rc2 is not None:
            nm.metric_list(ws, rc2, offsets, idx)
        s["x"], s["xb"] = s["xb"], s["x"]
        s["y"], s["yb"] = s["yb"], s["y"]
        s["t"], s["tb"] = s["tb"], s["t"]
        s["step"] += 1

    log(f"[bench] N={n} k={k} cell_w={cell_w} metric={'on' if rc2 else 'off'} "
        f"warmup={args.warmup} steps={args.steps}")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    if nm.check(ws) != 0:
        raise RuntimeError("device error during warmup")
    log("[bench] warmup done")

    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status = nm.check(ws)
    if status != 0:
        raise RuntimeError(f"device error in timed steps: {nm.nm.status_str(status)}")
    ms_step = (t1 - t0) * 1e3 / args.steps
    k_ms = sum(a.elapsed_time(b) for a, b in events) / args.steps
    log(f"[bench] timed {args.steps} steps: {ms_step:.4f} ms/step, fused kernel {k_ms:.4f} ms")

    value = n / (ms_step * 1e-3)
    bytes_per_ps = 24 + 4 * k
    achieved = bytes_per_ps * n / (k_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64/f64",
        "data": "synthetic",
        "config": {
            "workload": f"uniform N={n}, L=2^20, k={k} kNN rebuild + Eq.2 align + Eq.1 move"
                        + (f" + metric list r_c^2={rc2}" if rc2 is not None else "")
                        + ", v0=64, eta=0.2, Philox seed 0, every list rebuilt every step",
            "n": n, "k": k, "cell_w": cell_w, "box": box, "rc2": rc2,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_knn_align<{k}>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel_ms": k_ms,
            "bytes_per_particle_step": bytes_per_ps,
        },
        "step_roofline_frac": bytes_per_ps * n / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(x, y, th, k, rc2, box, args.cpu_seconds)
        log(f"[bench] cpu baseline {out['cpu_baseline']['value']:.3g} particle-steps/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
