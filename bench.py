"""Benchmark: iterated FP64 Smart Laplacian on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode all|single|batch|serve]
                    [--workload grid4096|annulus4096|grid1024] [--batch-meshes M] [--serve-rates R,...]

Headline (``value``): one step is one complete smoothing job through the C
ABI (``smooth_mesh_device``) on a 4096 x 4096 jittered grid (16.8M nodes,
33.5M triangles, random diagonals, +-0.4h jitter): validation, Hilbert
reordering, tile build, 100 Jacobi sweeps with the convergence test fused,
un-permuting -- from device-resident inputs to device-resident output.  Each
step starts from the same input coordinates (a device copy, inside the timed
region).  value = free nodes x sweeps x K / elapsed wall time.

roofline: the sweep kernel (the dominant kernel), algorithmic bytes per
launch (sum over free nodes of 36 + 4 d_i + 2 t_i) / its mean duration from
HIP events on the library's stream, against 8 TB/s.

batched: M independent jittered grids (side log-uniform in [24, 450],
random diagonals, +-0.35h, seeds 10000 + m), 50 sweeps each, smoothed by one
``sl_batch_smooth`` call (one work list, hipGraph-replayed sweep loop) and,
for comparison, by M plain ``smooth_mesh`` calls one after another.  Both
take host arrays in and give host arrays out.

serving: Poisson arrivals at each rate of smoothing requests (side
log-uniform in [32, 2048], random diagonals, +-0.4h; half of the requests
run 10-200 sweeps, half run to a 1e-8 displacement tolerance with a 10,000-sweep
cap) submitted to the continuous-batching server; latency is completion time
minus submission time.  The same arrival sequence is also served by a plain
loop that runs one ``smooth_mesh`` call at a time in arrival order.

cpu_baseline: the FP64 oracle, all host threads, on whole sweeps of the
headline mesh for about 10 s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import queue
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_KERNELS = {1: "k_sweep", 2: "k_sweep_tile"}
GEN_THREADS = 8


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


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
    for f in ("sl_tile_sweep.hip",):
        with open(os.path.join(ROOT, "paper_1502_00355_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(m, threads: int, seconds: float):
    """Whole Jacobi sweeps of the oracle on m with `threads` threads for about
    `seconds`: (node-updates/s, sweeps, elapsed)."""
    import oracle
    X = m.coords.copy()
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        X, _, _, _ = oracle.sweep(m, X, threads=threads)
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return m.n_interior * sweeps / el, sweeps, el


def cpu_baseline(m, seconds: float = 10.0):
    """The FP64 oracle on the host: all threads (the reported value) and one
    thread, each for about `seconds` of whole sweeps of the headline mesh."""
    import oracle
    threads = oracle.max_threads()
    v, sweeps, el = _oracle_rate(m, threads, seconds)
    v1, sweeps1, el1 = _oracle_rate(m, 1, seconds)
    free = m.n_interior
    return {"value": v, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d whole Jacobi sweeps of %s (%d free nodes) in %.1f s on %d threads" %
                      (sweeps, m.name, free, el, threads),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": v1, "unit": "node-updates/s", "cores": 1,
                              "sample": "%d whole Jacobi sweeps in %.1f s on 1 thread" % (sweeps1, el1)}}


def tile_opts(args):
    return {"tile_nodes": args.tile_nodes, "tile_wg_per_cu": args.wg_per_cu}


def converge_on(sl, torch, m, dev, X0, work, cap, tol=1e-9):
    """The mesh already on the device, run from its input positions until the
    largest displacement of a sweep is below tol (cap sweeps at most)."""
    work.copy_(X0)
    r = sl.smooth_mesh_device(work, *dev[1:], iterations=cap, tol=tol)
    torch.cuda.synchronize()
    log("converge %s: %d sweeps, last max |dx|^2 %.3e, %.1f ms of sweeps" %
        (m.name, r.iterations_run, r.max_disp_sq_last, r.sweep_ms))
    return {"workload": m.name, "tol": tol, "cap": cap, "iterations_run": r.iterations_run,
            "converged": r.iterations_run < cap, "max_disp_sq_last": r.max_disp_sq_last,
            "accepted_last": r.accepted_last, "sweep_ms": r.sweep_ms, "setup_ms": r.setup_ms,
            "sweep_node_updates_per_s": m.n_interior * r.iterations_run / (r.sweep_ms / 1e3)}


def run_single(args, sl, torch, name=None, steps=None, warmup=None, f32=None, autotune=None, converge=False):
    m, iters = workload(name or args.workload)
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    f32 = args.f32 if f32 is None else f32
    autotune = args.autotune if autotune is None else autotune
    free = m.n_interior
    alg_bytes = algorithmic_bytes(m)
    tuning = None
    if autotune:
        t = sl.autotune([m], layout=args.layout)
        tuning = t.as_dict()
        log("autotune: tile_nodes %d, wg/CU %d in %.0f ms" % (t.tile_nodes, t.tile_wg_per_cu, t.tune_ms))
    dev = sl.to_device(m, "cuda:0")
    X0 = dev[0].clone()
    work = torch.empty_like(X0)
    stream = torch.cuda.current_stream()
    log("workload %s: %d nodes, %d free, %d sweeps/step, alg bytes/sweep %d" %
        (m.name, m.n_nodes, free, iters, alg_bytes))

    def step():
        work.copy_(X0)
        return sl.smooth_mesh_device(work, *dev[1:], iterations=iters, layout=args.layout, reorder=args.reorder,
                                     kernel=args.kernel, stream=stream, **tile_opts(args))

    for w in range(warmup):
        r = step()
        log("warmup %d: setup %.2f ms, sweeps %.2f ms" % (w, r.setup_ms, r.sweep_ms))
    torch.cuda.synchronize()
    sweep_ms, setup_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
        sweep_ms.append(r.sweep_ms)
        setup_ms.append(r.setup_ms)
        assert r.iterations_run == iters
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log("timed %d steps of %s in %.3f s" % (steps, m.name, el))
    f32_out = None
    if f32:
        # the same job in single precision (the paper's precision), reported beside the FP64 headline
        f_sweep, f_t = [], []
        for k in range(steps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            work.copy_(X0)
            rf = sl.smooth_mesh_device(work, *dev[1:], iterations=iters, layout=args.layout, reorder=args.reorder,
                                       stream=stream, precision="f32", **tile_opts(args))
            torch.cuda.synchronize()
            if k:
                f_t.append(time.perf_counter() - t)
                f_sweep.append(rf.sweep_ms)
        f_sweep_s = float(np.mean(f_sweep)) / 1e3 / iters
        f_bytes = alg_bytes - 16 * free
        f32_out = {"ms_per_step": 1e3 * float(np.mean(f_t)), "node_updates_per_s": free * iters / float(np.mean(f_t)),
               "sweep_ms_per_sweep": f_sweep_s * 1e3, "sweep_only_node_updates_per_s": free / f_sweep_s,
               "alg_bytes_per_launch": f_bytes, "hbm_gbs_algorithmic": f_bytes / f_sweep_s / 1e9,
               "hbm_pct_peak": 100.0 * f_bytes / f_sweep_s / 1e9 / HBM_PEAK_GBS}
        log("f32: %.3f ms per sweep, %.1f%% of HBM peak" % (f_sweep_s * 1e3, f32_out["hbm_pct_peak"]))
    avg_sweep_s = float(np.mean(sweep_ms)) / 1e3 / iters
    achieved = alg_bytes / avg_sweep_s / 1e9
    out = {
        "metric": "node-updates/s",
        "value": free * iters * steps / el,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": el * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": m.name, "nodes": m.n_nodes, "free_nodes": free, "triangles": m.n_tris,
                   "sweeps_per_step": iters, "form": "jacobi", "layout": args.layout, "reorder": args.reorder,
                   "kernel": {1: "node", 2: "tile"}.get(r.kernel_used, "?"), "tile_nodes": r.tile_nodes},
        "autotune": tuning,
        "single_precision": f32_out,
        "sweep_only_node_updates_per_s": free / avg_sweep_s,
        "sweep_ms_per_sweep": avg_sweep_s * 1e3,
        "setup_ms_per_step": float(np.mean(setup_ms)),
        "hbm_gbs_algorithmic": achieved,
        "hbm_pct_peak": 100.0 * achieved / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": SWEEP_KERNELS.get(r.kernel_used, "?"), "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (traffic_from_profile(kernel_source_hash()) if m.name == "grid4096_random_j0.4_s3"
                                 else None),
                     "alg_bytes_per_launch": alg_bytes},
    }
    if converge:
        out["converge"] = converge_on(sl, torch, m, dev, X0, work, args.converge_cap)
    return out, m


KERNEL_NAMES = {1: "node", 2: "tile", 3: "resident", 4: "lanes"}


def run_form_b(args, sl, torch, m=None):
    """Form B (eq. (3): coloured, in place) on the 16.8M-node grid, 100
    sweeps per step as the headline's Form A, with the per-sweep time of the
    sweep kernel launches beside Form A's; then every sweep kernel the
    library has on the same mesh and job: Form A's tile kernel, the node
    kernel, the lane-group kernel at widths 4, 8 and 16, and Form B's
    automatic choice (the node kernel) beside its colour-class tiles."""
    if m is None:
        m, _ = workload("grid4096")
    iters, steps = 100, max(1, min(args.steps, 5))
    dev = sl.to_device(m, "cuda:0")
    X0 = dev[0].clone()
    work = torch.empty_like(X0)
    cases = [("form_b", "colored", {}), ("form_a", "jacobi", {}),
             ("form_b_class_tiles", "colored", {"kernel": "tile"}),
             ("form_a_node", "jacobi", {"kernel": "node"}),
             ("form_a_lanes4", "jacobi", {"kernel": "lanes", "lane_width": 4}),
             ("form_a_lanes8", "jacobi", {"kernel": "lanes", "lane_width": 8}),
             ("form_a_lanes16", "jacobi", {"kernel": "lanes", "lane_width": 16}),
             ("form_b_lanes4", "colored", {"kernel": "lanes", "lane_width": 4})]
    res = {}
    for name, form, kw in cases:
        best = None
        for k in range(steps + 1):
            work.copy_(X0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = sl.smooth_mesh_device(work, *dev[1:], iterations=iters, form=form, **kw)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            if k and (best is None or r.sweep_ms < best[1].sweep_ms):
                best = (el, r)
        el, r = best
        res[name] = {"ms_per_step": el * 1e3, "sweep_ms_per_sweep": r.sweep_ms / iters, "setup_ms": r.setup_ms,
                     "kernel": KERNEL_NAMES.get(r.kernel_used, "?"), "colors": r.n_colors,
                     "sweep_node_updates_per_s": m.n_interior * iters / (r.sweep_ms / 1e3)}
        if kw.get("lane_width"):
            res[name]["lane_width"] = kw["lane_width"]
        log("%s: %.4f ms per sweep (%s kernel, %d colours), setup %.2f ms" %
            (name, r.sweep_ms / iters, res[name]["kernel"], r.n_colors, r.setup_ms))
    return {"workload": m.name, "sweeps": iters, "form_b": res["form_b"], "form_a": res["form_a"],
            "b_over_a_sweep_time": res["form_b"]["sweep_ms_per_sweep"] / res["form_a"]["sweep_ms_per_sweep"],
            "kernels": {k: v for k, v in res.items() if k not in ("form_a", "form_b")}}


def run_layouts(args, sl, torch):
    """The 1024 x 1024 permuted grid (100 sweeps) in AoS and SoA, with and
    without the Hilbert reorder: sweep-loop rate of each."""
    import meshgen
    m = meshgen.permute_mesh(meshgen.make_grid(1024, "random", 0.4, 2), 2)
    dev = sl.to_device(m, "cuda:0")
    X0 = dev[0].clone()
    work = torch.empty_like(X0)
    rows = []
    for layout in ("aos", "soa"):
        for reorder in ("none", "hilbert"):
            best = None
            for _ in range(3):
                work.copy_(X0)
                r = sl.smooth_mesh_device(work, *dev[1:], iterations=100, layout=layout, reorder=reorder)
                best = r if best is None or r.sweep_ms < best.sweep_ms else best
            rows.append({"layout": layout, "reorder": reorder, "kernel": {1: "node", 2: "tile"}[best.kernel_used],
                         "sweep_ms_per_sweep": best.sweep_ms / 100,
                         "sweep_node_updates_per_s": m.n_interior * 100 / (best.sweep_ms / 1e3),
                         "setup_ms": best.setup_ms})
            log("grid1024 %s/%s: %.4f ms per sweep" % (layout, reorder, best.sweep_ms / 100))
    return {"workload": "grid1024_random_j0.4_s2_permuted", "free_nodes": m.n_interior, "sweeps": 100,
            "variants": rows}


def run_converge(args, sl, torch):
    """The headline mesh run until the largest displacement of a sweep is
    below 1e-9 (cap 100,000 sweeps): the sweep count it takes."""
    m, _ = workload(args.workload)
    dev = sl.to_device(m, "cuda:0")
    r = sl.smooth_mesh_device(*dev, iterations=args.converge_cap, tol=1e-9)
    torch.cuda.synchronize()
    log("converge %s: %d sweeps, last max |dx|^2 %.3e, %.1f s of sweeps" %
        (m.name, r.iterations_run, r.max_disp_sq_last, r.sweep_ms / 1e3))
    return {"workload": m.name, "tol": 1e-9, "cap": args.converge_cap, "iterations_run": r.iterations_run,
            "converged": r.iterations_run < args.converge_cap, "max_disp_sq_last": r.max_disp_sq_last,
            "accepted_last": r.accepted_last, "sweep_ms": r.sweep_ms,
            "sweep_node_updates_per_s": m.n_interior * r.iterations_run / (r.sweep_ms / 1e3)}


def run_paper(args, sl, torch):
    """Meshes like the paper's (Sec. 4, Tables 6-9): Delaunay meshes of
    1K-100K uniformly random points.  Two runs of each: 100 sweeps of Form A
    (AoS and SoA) and Form B (and, on meshes small enough, both forms on the
    resident kernel); and each form run to convergence (largest displacement
    of a sweep below 1e-9, cap 100,000 sweeps) -- the paper compares the
    forms to convergence (Sec. 5.2) but states neither its criterion nor its
    sweep counts.  GPU time is the whole smooth_mesh call (host arrays in and
    out) and, separately, the sweep loop; the oracle runs the same work on one
    host thread, as the paper compares against one CPU core.  The paper used
    FP32 on a GT640: its numbers are context only."""
    import meshgen
    import oracle
    tol, cap = 1e-9, 100000
    rows = []

    def gpu_best(m, iters, tol_, opts):
        best = None
        for _ in range(3):
            t = time.perf_counter()
            _, r, _ = sl.smooth_mesh(m.coords, m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary,
                                     iters, tol_, **opts)
            el = (time.perf_counter() - t) * 1e3
            best = (el, r) if best is None or el < best[0] else best
        return best

    for n in (1000, 5000, 10000, 50000, 100000):
        m = meshgen.make_delaunay(n, 11)
        row = {"points": n, "free_nodes": m.n_interior, "triangles": m.n_tris}
        variants = [("A_aos", {}), ("A_soa", {"layout": "soa"}), ("B_aos", {"form": "colored"}),
                    ("B_soa", {"form": "colored", "layout": "soa"})]
        if m.n_nodes <= 2048:        # the resident kernel (opt-in) holds meshes of about this size
            variants += [("A_resident", {"kernel": "resident"}), ("B_resident", {"form": "colored", "kernel": "resident"})]
        for label, opts in variants:
            el, r = gpu_best(m, 100, 0.0, opts)
            row["gpu_" + label + "_ms"] = el
            row["gpu_" + label + "_sweep_ms"] = r.sweep_ms
        for label, form in (("A", "jacobi"), ("B", "colored")):
            t = time.perf_counter()
            oracle.smooth(m, 100, threads=1, want_flags=False, form=form)
            row["cpu_" + label + "_ms"] = (time.perf_counter() - t) * 1e3
        row["speedup_A_aos"] = row["cpu_A_ms"] / row["gpu_A_aos_ms"]
        row["speedup_B_aos"] = row["cpu_B_ms"] / row["gpu_B_aos_ms"]
        # to convergence
        for label, opts in (("A_aos", {}), ("A_soa", {"layout": "soa"}), ("B_aos", {"form": "colored"}),
                            ("B_soa", {"form": "colored", "layout": "soa"})):
            el, r = gpu_best(m, cap, tol, opts)
            row["conv_gpu_" + label + "_ms"] = el
            row["conv_gpu_" + label + "_sweep_ms"] = r.sweep_ms
            row["iterations_" + label] = r.iterations_run
        for label, form in (("A", "jacobi"), ("B", "colored")):
            t = time.perf_counter()
            ref = oracle.smooth(m, cap, tol=tol, threads=1, want_flags=False, form=form)
            row["conv_cpu_" + label + "_ms"] = (time.perf_counter() - t) * 1e3
            row["conv_cpu_iterations_" + label] = ref.iterations_run
        row["iterations_A"] = row["iterations_A_aos"]
        row["iterations_B"] = row["iterations_B_aos"]
        row["conv_speedup_A_aos"] = row["conv_cpu_A_ms"] / row["conv_gpu_A_aos_ms"]
        row["conv_speedup_B_aos"] = row["conv_cpu_B_ms"] / row["conv_gpu_B_aos_ms"]
        log("paper mesh %d: 100 sweeps GPU A %.2f ms (sweeps %.2f), CPU A %.0f ms; to 1e-9: A %d sweeps %.2f ms, "
            "B %d sweeps %.2f ms (CPU A %.0f ms, B %.0f ms)" %
            (n, row["gpu_A_aos_ms"], row["gpu_A_aos_sweep_ms"], row["cpu_A_ms"], row["iterations_A"],
             row["conv_gpu_A_aos_ms"], row["iterations_B"], row["conv_gpu_B_aos_ms"], row["conv_cpu_A_ms"],
             row["conv_cpu_B_ms"]))
        rows.append(row)
    return {"workload": "delaunay_uniform_points_1K-100K_s11", "sweeps": 100, "converge_tol": tol,
            "converge_cap": cap, "dtype": "f64", "cpu_threads": 1, "rows": rows}


def gen_meshes(specs):
    """specs: list of (side, diag, jitter, seed); generated on host threads."""
    import meshgen
    with ThreadPoolExecutor(GEN_THREADS) as ex:
        return list(ex.map(lambda s: meshgen.make_grid(int(s[0]), s[1], s[2], int(s[3])), specs))


def run_batch(args, sl):
    """Batched (one sl_batch_smooth call) against plain per-mesh calls."""
    import meshgen
    M, iters = args.batch_meshes, 50
    sides = meshgen.batch_sides(M, 24, 450, 10000)
    t = time.perf_counter()
    meshes = gen_meshes([(s, "random", 0.35, 10000 + i) for i, s in enumerate(sides)])
    free = sum(m.n_interior for m in meshes)
    nodes = sum(m.n_nodes for m in meshes)
    log("batch: %d meshes, %d nodes, %d free, generated in %.1f s" % (M, nodes, free, time.perf_counter() - t))
    tuning = None
    if args.autotune:
        t = sl.autotune(meshes)
        tuning = t.as_dict()
        log("autotune: tile_nodes %d, wg/CU %d in %.0f ms" % (t.tile_nodes, t.tile_wg_per_cu, t.tune_ms))
    sl.batch_smooth(meshes[: min(M, 8)], iters)          # warm-up (code objects, memory pool)
    t = time.perf_counter()
    _, reps, br = sl.batch_smooth(meshes, iters)
    el_b = time.perf_counter() - t
    assert all(r.iterations_run == iters for r in reps)
    log("batched: %.3f s (setup %.1f ms, graph %.1f ms, sweeps %.1f ms, results %.1f ms)" %
        (el_b, br.setup_ms, br.graph_ms, br.sweep_ms, br.results_ms))
    # the same batch again: the library's device blocks are now cached, as
    # for a caller that smooths batches one after another
    t = time.perf_counter()
    _, _, br2 = sl.batch_smooth(meshes, iters)
    el_b2 = time.perf_counter() - t
    log("batched again: %.3f s (setup %.1f ms, results %.1f ms)" % (el_b2, br2.setup_ms, br2.results_ms))
    upd = free * iters
    out = {
        "workload": "batch%d_grids_side24-450_random_j0.35_seeds10000+" % M,
        "meshes": M, "nodes": nodes, "free_nodes": free, "sweeps": iters,
        "batched_node_updates_per_s": upd / el_b, "batched_s": el_b,
        "batched_setup_ms": br.setup_ms, "batched_graph_ms": br.graph_ms, "batched_sweep_ms": br.sweep_ms,
        "batched_results_ms": br.results_ms,
        "batched_sweep_node_updates_per_s": upd / (br.sweep_ms / 1e3),
        "batched_repeat_s": el_b2, "batched_repeat_setup_ms": br2.setup_ms,
        "tiles": br.tiles, "graph_used": bool(br.graph_used), "autotune": tuning,
    }
    if not args.plain:
        return out
    plain_sweep_ms = 0.0
    t = time.perf_counter()
    for m in meshes:
        _, rep, _ = sl.smooth_mesh(m.coords, m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary, iters)
        plain_sweep_ms += rep.sweep_ms
    el_p = time.perf_counter() - t
    log("plain: %.3f s (sweeps %.1f ms)" % (el_p, plain_sweep_ms))
    out.update({
        "plain_node_updates_per_s": upd / el_p, "plain_s": el_p, "plain_sweep_ms": plain_sweep_ms,
        "plain_sweep_node_updates_per_s": upd / (plain_sweep_ms / 1e3),
        "speedup_whole_job": el_p / el_b, "speedup_sweeps": plain_sweep_ms / br.sweep_ms,
        "speedup_whole_job_repeat": el_p / el_b2,
    })
    return out


def serve_requests(rate, count, pool, rng):
    """(arrival offsets, pool index, iterations, tol) for one Poisson run."""
    gaps = rng.exponential(1.0 / rate, size=count)
    arr = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(count):
        idx = int(rng.integers(len(pool)))
        if rng.random() < 0.5:
            reqs.append((float(arr[k]), idx, int(rng.integers(10, 201)), 0.0))
        else:
            reqs.append((float(arr[k]), idx, 10000, 1e-8))
    return reqs


def _pct(v, p):
    return float(np.percentile(np.asarray(v), p)) * 1e3 if len(v) else None


def serve_server(sl, pool, reqs):
    """Submits each request at its arrival time.  Latency runs from the
    scheduled arrival to the result on the host: the server's own
    completion-minus-submission time plus however late the submission
    itself was (a submit that waits for the server counts against it)."""
    with sl.Server() as S:
        t0 = time.perf_counter()
        ids, late = [], []
        for (at, idx, it, tol) in reqs:
            d = t0 + at - time.perf_counter()
            if d > 0:
                time.sleep(d)
            m = pool[idx]
            late.append(time.perf_counter() - (t0 + at))
            ids.append(S.submit(m, it, tol))
        lat, upd = [], 0
        first, last = None, None
        for rid, lt, (at, idx, it, tol) in zip(ids, late, reqs):
            r = S.wait(rid, timeout=300.0)
            if r.status != sl.SL_OK:
                raise RuntimeError("request failed: " + r.message)
            lat.append(lt + r.times.done_s - r.times.submitted_s)
            upd += pool[idx].n_interior * r.report.iterations_run
            first = r.times.submitted_s - lt if first is None else min(first, r.times.submitted_s - lt)
            last = r.times.done_s if last is None else max(last, r.times.done_s)
        st = S.stats()
    return lat, upd, last - first, st


def serve_plain(sl, pool, reqs):
    """One smooth_mesh call at a time, in arrival order; latency from the
    scheduled arrival to the result on the host."""
    q = queue.Queue()
    lat = [None] * len(reqs)
    upd = [0]
    t0 = time.perf_counter()

    def worker():
        while True:
            k = q.get()
            if k is None:
                return
            at, idx, it, tol = reqs[k]
            m = pool[idx]
            _, rep, _ = sl.smooth_mesh(m.coords, m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.tris, m.boundary, it, tol)
            lat[k] = time.perf_counter() - (t0 + at)
            upd[0] += m.n_interior * rep.iterations_run

    th = threading.Thread(target=worker)
    th.start()
    for k, (at, idx, it, tol) in enumerate(reqs):
        d = t0 + at - time.perf_counter()
        if d > 0:
            time.sleep(d)
        q.put(k)
    q.put(None)
    th.join()
    return lat, upd[0], time.perf_counter() - t0


def run_serve(args, sl):
    import meshgen
    P = args.serve_pool
    sides = meshgen.batch_sides(P, 32, 2048, 20000)
    t = time.perf_counter()
    pool = gen_meshes([(s, "random", 0.4, 20000 + i) for i, s in enumerate(sides)])
    log("serve: pool of %d meshes (%d nodes in total) generated in %.1f s" %
        (P, sum(m.n_nodes for m in pool), time.perf_counter() - t))
    rng = np.random.Generator(np.random.PCG64(30000))
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    # warm-up: one small request through each path
    small = min(range(P), key=lambda i: pool[i].n_nodes)
    serve_server(sl, pool, [(0.0, small, 10, 0.0)])
    serve_plain(sl, pool, [(0.0, small, 10, 0.0)])
    rows = []
    for rate in rates:
        # serve_max_requests arrivals, or as many as arrive in serve_seconds
        # at the low rates
        count = int(min(args.serve_max_requests, max(60, rate * args.serve_seconds)))
        reqs = serve_requests(rate, count, pool, rng)
        lat, upd, span, st = serve_server(sl, pool, reqs)
        log("serve rate %g: %d requests, server p50 %.1f ms p99 %.1f ms, %.3g node-updates/s" %
            (rate, count, _pct(lat, 50), _pct(lat, 99), upd / span))
        plat, pupd, pspan = serve_plain(sl, pool, reqs)
        log("serve rate %g: plain p50 %.1f ms p99 %.1f ms, %.3g node-updates/s" %
            (rate, _pct(plat, 50), _pct(plat, 99), pupd / pspan))
        rows.append({"rate_req_per_s": rate, "requests": count,
                     "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "node_updates_per_s": upd / span,
                     "plain_p50_ms": _pct(plat, 50), "plain_p99_ms": _pct(plat, 99),
                     "plain_node_updates_per_s": pupd / pspan, "server_steps": st.steps})
    return {"workload": "serve_grids_side32-2048_random_j0.4_pool%d" % P,
            "requests_mix": "half 10-200 sweeps, half tol 1e-8 (cap 10000)",
            "latency": "scheduled arrival to the result on the host", "rates": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="all",
                    choices=["all", "single", "formb", "layouts", "paper", "batch", "serve", "converge"])
    ap.add_argument("--workload", default="grid4096")
    ap.add_argument("--layout", default="aos")
    ap.add_argument("--reorder", default="hilbert")
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--tile-nodes", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false")
    ap.add_argument("--no-f32", dest="f32", action="store_false")
    ap.add_argument("--batch-meshes", type=int, default=10000)
    ap.add_argument("--no-plain", dest="plain", action="store_false",
                    help="batch mode: skip the separate-calls comparison")
    ap.add_argument("--converge-cap", type=int, default=100000)
    ap.add_argument("--serve-rates", default="10,30,100,300,1000,2000")
    ap.add_argument("--serve-pool", type=int, default=48)
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="arrivals of one rate span at most this long (the low rates)")
    ap.add_argument("--serve-max-requests", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the smoothing path runs on a single MI355X (the multi-GPU "
              "split is a design, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1502_00355_amd as sl

    torch.cuda.set_device(0)
    out, m = {}, None
    if args.mode in ("all", "single"):
        out, m = run_single(args, sl, torch, converge=args.mode == "all")
    if args.mode == "all":
        # the annulus variant of the 16.8M-node mesh: 100 timed sweeps per
        # step as for the headline, then its run to tol 1e-9
        an, _ = run_single(args, sl, torch, name="annulus4096", steps=min(args.steps, 10), warmup=1, f32=False,
                           autotune=False, converge=True)
        out["annulus"] = {k: an[k] for k in ("value", "unit", "ms_per_step", "steps", "config", "sweep_ms_per_sweep",
                                              "sweep_only_node_updates_per_s", "setup_ms_per_step",
                                              "hbm_gbs_algorithmic", "hbm_pct_peak", "roofline", "converge")}
    if args.mode in ("all", "formb"):
        out["form_b"] = run_form_b(args, sl, torch, m)
    if args.mode == "converge":
        out["converge"] = run_converge(args, sl, torch)
    if args.mode in ("all", "layouts"):
        out["layouts"] = run_layouts(args, sl, torch)
    if args.mode in ("all", "paper"):
        out["paper_tables"] = run_paper(args, sl, torch)
    if args.mode in ("all", "batch"):
        out["batched"] = run_batch(args, sl)
    if args.mode in ("all", "serve"):
        out["serving"] = run_serve(args, sl)
    if m is not None and not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
