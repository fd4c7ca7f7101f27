"""Benchmark: iterated FP64 Smart Laplacian on a 16.8M-node mesh, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload grid4096|annulus4096|grid1024]

A step is one complete smoothing job through the C ABI
(``smooth_mesh_device``): validation, Hilbert reordering, relabelling, fan
build, 100 Jacobi sweeps with the convergence test fused, un-permuting --
from device-resident inputs to device-resident output.  Each step starts from
the same input coordinates (a device copy, inside the timed region).

value: node-updates/s = free nodes x sweeps x K / elapsed wall time.
roofline: the sweep kernel (the dominant kernel), algorithmic bytes per
launch (sum over free nodes of 36 + 4 d_i + 2 t_i) / its mean duration from
HIP events on the library's stream, against 8 TB/s.
cpu_baseline: the FP64 oracle, all host threads, on whole sweeps of the same
mesh for about 10 s.
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

HBM_PEAK_GBS = 8000.0
SWEEP_KERNELS = {1: "k_sweep", 2: "k_sweep_tile"}


def workload(name: str):
    import meshgen
    if name == "grid4096":
        return meshgen.make_grid(4096, "random", 0.4, 3, name="grid4096_random_j0.4_s3"), 100
    if name == "annulus4096":
        return meshgen.make_annulus(4096, 4096, seed=4, name="annulus4096x4096_random_j0.4_s4"), 100
    if name == "grid1024":
        m = meshgen.permute_mesh(meshgen.make_grid(1024, "random", 0.4, 2), 2)
        return m, 100
    raise SystemExit("unknown workload " + name)


def algorithmic_bytes(m) -> int:
    """Sum over free nodes of 16 (read x_i) + 16 (write x_i) + 4 (row
    offset) + 4 d_i (neighbour ids) + 2 t_i (fan entries)."""
    free = m.boundary == 0
    d = np.diff(m.nbr_ptr.astype(np.int64))[free]
    t = np.diff(m.tri_ptr.astype(np.int64))[free]
    return int(np.sum(36 + 4 * d + 2 * t))


def traffic_from_profile(kernel_source_hash: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "sweep_grid4096_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("sl_sweep.hip", "sl_tiles.hip", "sl_common.h"):
        with open(os.path.join(ROOT, "paper_1502_00355_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(m, seconds: float = 10.0):
    import oracle
    threads = oracle.max_threads()
    X = m.coords.copy()
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        X, _, _, _ = oracle.sweep(m, X, threads=threads)
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    free = int(np.count_nonzero(m.boundary == 0))
    return {"value": free * sweeps / el, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d whole Jacobi sweeps of %s (%d free nodes) in %.1f s" % (sweeps, m.name, free, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid4096")
    ap.add_argument("--layout", default="aos")
    ap.add_argument("--reorder", default="hilbert")
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the smoothing path on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1502_00355_amd as sl

    torch.cuda.set_device(0)
    m, iters = workload(args.workload)
    free = m.n_interior
    alg_bytes = algorithmic_bytes(m)
    dev = sl.to_device(m, "cuda:0")
    X0 = dev[0].clone()
    work = torch.empty_like(X0)
    stream = torch.cuda.current_stream()
    print("# workload %s: %d nodes, %d free, %d sweeps/step, alg bytes/sweep %d" %
          (m.name, m.n_nodes, free, iters, alg_bytes), file=sys.stderr, flush=True)

    def step():
        work.copy_(X0)
        return sl.smooth_mesh_device(work, *dev[1:], iterations=iters, layout=args.layout, reorder=args.reorder,
                                     kernel=args.kernel, stream=stream)

    for w in range(args.warmup):
        r = step()
        print("# warmup %d: setup %.2f ms, sweeps %.2f ms" % (w, r.setup_ms, r.sweep_ms), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sweep_ms, setup_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        sweep_ms.append(r.sweep_ms)
        setup_ms.append(r.setup_ms)
        assert r.iterations_run == iters
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    value = free * iters * args.steps / el
    avg_sweep_s = float(np.mean(sweep_ms)) / 1e3 / iters
    achieved = alg_bytes / avg_sweep_s / 1e9
    traffic = traffic_from_profile(kernel_source_hash())
    out = {
        "metric": "node-updates/s",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": m.name, "nodes": m.n_nodes, "free_nodes": free, "triangles": m.n_tris,
                   "sweeps_per_step": iters, "form": "jacobi", "layout": args.layout, "reorder": args.reorder,
                   "kernel": {1: "node", 2: "tile"}.get(r.kernel_used, "?")},
        "sweep_only_node_updates_per_s": free / avg_sweep_s,
        "sweep_ms_per_sweep": avg_sweep_s * 1e3,
        "setup_ms_per_step": float(np.mean(setup_ms)),
        "hbm_gbs_algorithmic": achieved,
        "hbm_pct_peak": 100.0 * achieved / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": SWEEP_KERNELS.get(r.kernel_used, "?"), "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
