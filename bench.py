#!/usr/bin/env python3
"""Benchmark: reverse-mode gradient of the FP64 element objective on a 128^3
structured hex mesh (2,097,152 nodes, 2,048,383 eight-node elements) on one
MI355X.

A step is one pg_gradient call (forward gather + psi + reduction + seeded
reverse scatter) on one mesh.  Three copies of the mesh (~690 MB, more than
the 256 MB last-level cache) are used in rotation so every step streams its
inputs from HBM.  The objective alone is timed the same way for the
gradient/objective time ratio.

Prints one JSON line (rank 0).  --gpus above 1 is refused: this benchmark
measures one GPU's throughput.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak, GB/s

# Algorithmic bytes of the 128^3 FP64 workload: every input read once, every
# output written once, the gathers counted at perfect node reuse.
#   conn 2,048,383 x 8 x 4 B + B 2,048,383 x 8 x 8 B + w 2,048,383 x 8 B
#   + x 2,097,152 x 8 B (+ grad 2,097,152 x 8 B for the gradient)
def algorithmic_bytes(n_nodes: int, n_elems: int, k: int, esz: int, gradient: bool) -> int:
    b = n_elems * k * 4 + n_elems * k * esz + n_elems * esz + n_nodes * esz
    return b + (n_nodes * esz if gradient else 0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--side", type=int, default=128, help="nodes per axis of the hex mesh")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--adjoint", default="atomic", choices=["atomic", "gather", "colour", "tiled"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--copies", type=int, default=3, help="rotating input copies")
    ap.add_argument("--scatter", type=int, default=0, help="0 combine in LDS, 1 direct atomics")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 keys of the hex line")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the dense and batched-dense summaries of the hex line")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-per-instance keys of the hex line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", default="hex",
                    choices=["hex", "dense", "bdense", "batch", "chain", "paper", "program"],
                    help="hex (default, the headline), dense, bdense, batch, chain, paper, "
                         "program")
    ap.add_argument("--dense-n", type=int, default=10_000)
    ap.add_argument("--bd-m", type=int, default=4096)
    ap.add_argument("--bd-n", type=int, default=1024)
    ap.add_argument("--batch-n", type=int, default=256)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 512 MiB device copy (scale for byte counters)")
    return ap.parse_args()


# What the library's event hook times per gradient call, by adjoint schedule:
# one kernel for the atomic scatter, the range of the call's kernels otherwise.
HEX_KERNELS = {
    "atomic": "k_mesh_elem (gradient, atomic scatter with LDS combining)",
    "gather": "k_mesh_elem + k_mesh_node_gather (range)",
    "colour": "k_mesh_elem colour passes (range)",
    "tiled": "k_mesh_tiled + k_node_tiled (range)",
}


def traffic_record(kernel_key: str):
    """HBM bytes per launch of the dominant kernel, measured with rocprofv3
    byte counters (profiles/traffic.json), or None if the kernel sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        p = os.path.join(ROOT, src)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """The host's CPU model (/proc/cpuinfo) and its core counts."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "nproc": avail, "os_cpu_count": os.cpu_count()}


def _median_runs(fn, budget_s: float):
    import numpy as np
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        r = fn()
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end and len(times) >= 3:
            break
    return float(np.median(times)), len(times), r


def cpu_baseline(m, budget_s: float, gbytes: float):
    """The oracle's FP64 gradient of the whole mesh on the host: the OpenMP
    build on every core the process may use (the reported value) and the
    plain single-threaded build, each for half the budget."""
    import oracle
    med1, n1, _ = _median_runs(lambda: oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x),
                               budget_s / 2)
    medT, nT, r = _median_runs(
        lambda: oracle.mesh_gradient_threads(m.n_nodes, m.conn, m.B, m.w, m.x), budget_s / 2)
    threads = r[2]
    cpu = host_cpu()
    return {"value": round(gbytes / medT, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"full {m.name} FP64 gradient (f and grad), C oracle built with OpenMP on "
                      f"{threads} threads (per-thread partials combined in thread order), "
                      f"median of {nT} runs = {medT * 1e3:.1f} ms",
            "single_thread": {"value": round(gbytes / med1, 3), "unit": "GB/s", "cores": 1,
                              "sample": f"plain C oracle, median of {n1} runs = {med1 * 1e3:.1f} ms"},
            "cpu": cpu["model"], "nproc": cpu["nproc"], "os_cpu_count": cpu["os_cpu_count"]}


def bench_hex(args):
    import numpy as np
    import torch
    from paper_2507_13204_amd import MeshObjective, inputs

    dev = torch.device("cuda:0")
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    esz = 8 if args.dtype == "f64" else 4

    m = inputs.hex_mesh(args.side)
    conn = torch.from_numpy(m.conn).to(dev)
    B = torch.from_numpy(m.B).to(dev, tdt)
    w = torch.from_numpy(m.w).to(dev, tdt)
    x = torch.from_numpy(m.x).to(dev, tdt)
    copies = []
    for c in range(max(1, args.copies)):
        cc = (conn, B, w, x) if c == 0 else tuple(t.clone() for t in (conn, B, w, x))
        obj = MeshObjective(cc[0], cc[1], cc[2], m.n_nodes, adjoint=args.adjoint,
                            block=args.block, tile=args.tile, scatter=args.scatter)
        copies.append((obj, cc[3], torch.empty_like(cc[3]),
                       torch.empty((), dtype=torch.float64, device=dev)))
    torch.cuda.synchronize()

    def step(kind, i, rotate=True):
        obj, xx, g, f = copies[i % len(copies) if rotate else 0]
        if kind == "grad":
            obj.gradient(xx, out=g)
        else:
            obj.objective(xx)

    def run(kind: str, steps: int, warmup: int, rotate: bool = True):
        """ms per step over exactly `steps` back-to-back steps, then (in a
        second, separately timed pass) the average duration of the dominant
        kernel from the library's event hook."""
        for i in range(warmup):
            step(kind, i, rotate)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for i in range(steps):
            step(kind, i, rotate)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        for obj, *_ in copies:
            obj.timing(1)
        for i in range(steps):
            step(kind, i, rotate)
        torch.cuda.synchronize()
        kms, kn = 0.0, 0
        for obj, *_ in copies:
            a, b = obj.timing_read()
            obj.timing(0)
            kms += a
            kn += b
        return ms, kms / max(kn, 1)

    ms_grad, kms_grad = run("grad", args.steps, args.warmup)
    ms_obj, kms_obj = run("obj", args.steps, args.warmup)
    ms_grad_warm, _ = run("grad", args.steps, 2, rotate=False)

    gbytes = algorithmic_bytes(m.n_nodes, m.n_elems, 8, esz, True) / 1e9
    obytes = algorithmic_bytes(m.n_nodes, m.n_elems, 8, esz, False) / 1e9
    value = gbytes / (ms_grad * 1e-3)
    achieved = gbytes / (kms_grad * 1e-3)
    kernel_key = f"mesh_grad_{args.adjoint}_{args.dtype}_hex{args.side}"
    traffic = traffic_record(kernel_key)

    out = {
        "metric": "gradient GB/s & gradient/primal time ratio (FP64, 128^3 hex mesh), % HBM peak",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_grad, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded: x~U(-1,1), B~N(0,1), w~U(0.5,1.5), lexicographic hex connectivity)",
        "config": {"workload": f"hex mesh {args.side}^3 nodes, {m.n_elems} 8-node elements, "
                               f"{args.dtype} gradient, {args.adjoint} adjoint",
                   "n_nodes": m.n_nodes, "n_elems": m.n_elems, "k": 8,
                   "input_copies_rotated": len(copies)},
        "gradient_over_objective": round(ms_grad / ms_obj, 4),
        "objective_ms": round(ms_obj, 5),
        "objective_GBps": round(obytes / (ms_obj * 1e-3), 2),
        "pct_hbm_peak": round(100.0 * value / PEAK_HBM_GBS, 2),
        "warm_cache_GBps": round(gbytes / (ms_grad_warm * 1e-3), 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": HEX_KERNELS[args.adjoint],
                     "kernel_ms": round(kms_grad, 5),
                     "algorithmic_bytes": int(gbytes * 1e9)},
    }

    # the other derivative modes on the same mesh (tangent and Hessian-vector product)
    obj0, x0 = copies[0][0], copies[0][1]
    dvec = torch.ones_like(x0)
    hv = torch.empty_like(x0)
    out["hvp_ms"] = round(_timed(lambda: obj0.hvp(x0, dvec, out=hv), 20, 3), 5)
    out["jvp_ms"] = round(_timed(lambda: obj0.jvp(x0, dvec), 20, 3), 5)

    if args.dtype == "f64":
        import oracle
        f0, g0 = copies[0][0].gradient(copies[0][1])
        f_ref, g_ref = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
        gh = g0.cpu().numpy()
        out["error_vs_oracle"] = {
            "f": abs(f0.item() - f_ref) / abs(f_ref),
            "grad": float(np.linalg.norm(gh - g_ref) / np.linalg.norm(g_ref))}
    _progress("headline done")

    ccs = [(obj.conn, obj.B, obj.w, xx) for obj, xx, _, _ in copies]
    out["autograd"] = _hex_autograd(args, m, ccs)
    _progress("autograd done")
    if not args.no_variants:
        out["variants"] = _hex_variants(args, m, ccs, gbytes, ms_obj)
        _progress("variants done")
    if args.dtype == "f64" and not args.no_fp32:
        out["fp32"] = _hex_fp32(args, m)
        _progress("fp32 done")
    if not args.no_batch:
        out["batch"] = _batch_vs_per_instance(args)
        _progress("batch done")
    if not args.no_other:
        out.update(_other_configs(args))
        out.update(_small_sweeps(args))
        _progress("dense, batched dense and the small sweeps done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_seconds, gbytes)

    print(json.dumps(out), flush=True)


def _progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _rotating(fn, n_copies, steps, warmup):
    """ms per step of fn(i) over copies i mod n_copies, back to back."""
    import torch
    for i in range(warmup):
        fn(i % n_copies)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        fn(i % n_copies)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def _hex_autograd(args, m, ccs):
    """The autograd form on the rotating copies, for each policy of what the
    forward keeps: forward (grad mode off: the objective alone), forward with
    the gradient requested, and forward + backward, as a user of MeshFn sees
    them (host autograd overhead included)."""
    import torch
    from paper_2507_13204_amd import MeshFn, MeshObjective
    res = {}
    for pol in ("gradient", "store", "recompute"):
        objs = [MeshObjective(c, B, w, m.n_nodes, autograd=pol) for c, B, w, _ in ccs]
        xs = [x.detach().clone().requires_grad_(True) for *_, x in ccs]

        def fwd_nograd(i):
            with torch.no_grad():
                MeshFn.apply(xs[i], objs[i])

        def fwd(i):
            MeshFn.apply(xs[i], objs[i])

        def fwd_bwd(i):
            xs[i].grad = None
            MeshFn.apply(xs[i], objs[i]).backward()

        t0 = _rotating(fwd_nograd, len(objs), args.steps, 3)
        t1 = _rotating(fwd, len(objs), args.steps, 3)
        t2 = _rotating(fwd_bwd, len(objs), args.steps, 3)
        res[pol] = {"forward_nograd_ms": round(t0, 5), "forward_ms": round(t1, 5),
                    "forward_backward_ms": round(t2, 5),
                    "fwd_plus_bwd_over_fwd": round(t2 / t1, 4),
                    "fwd_plus_bwd_over_objective": round(t2 / t0, 4),
                    "cache": f"cold ({len(objs)} rotating copies)"}
        for o in objs:
            o.close()
    auto = MeshObjective(*ccs[0][:3], m.n_nodes)
    res["auto_policy"] = auto.autograd_policy
    auto.close()
    return res


def _hex_variants(args, m, ccs, gbytes, ms_obj):
    """The deterministic adjoint schedules on the rotating copies."""
    from paper_2507_13204_amd import MeshObjective
    import torch
    res = {}
    for adj in ("atomic", "gather", "colour", "tiled"):
        if adj == args.adjoint:
            continue
        objs = [MeshObjective(c, B, w, m.n_nodes, adjoint=adj) for c, B, w, _ in ccs]
        gs = [torch.empty_like(x) for *_, x in ccs]
        vms = _rotating(lambda i: objs[i].gradient(ccs[i][3], out=gs[i]), len(objs), args.steps, 3)
        res[adj] = {"ms": round(vms, 5), "GBps_algorithmic": round(gbytes / (vms * 1e-3), 2),
                    "over_objective": round(vms / ms_obj, 4),
                    "cache": f"cold ({len(objs)} rotating copies)"}
        for o in objs:
            o.close()
    return res


def _hex_fp32(args, m):
    """FP32 storage (x, B, w, grad), every accumulation FP64: time on rotating
    copies, algorithmic GB/s, and the error against the oracle run on the
    FP32-rounded inputs (the acceptance bar, 1e-5) and on the FP64 inputs."""
    import numpy as np
    import torch
    import oracle
    from paper_2507_13204_amd import MeshObjective
    dev = torch.device("cuda:0")
    conn = torch.from_numpy(m.conn).to(dev)
    B = torch.from_numpy(m.B).to(dev, torch.float32)
    w = torch.from_numpy(m.w).to(dev, torch.float32)
    x = torch.from_numpy(m.x).to(dev, torch.float32)
    cps = []
    for c in range(max(1, args.copies)):
        cc = (conn, B, w, x) if c == 0 else tuple(t.clone() for t in (conn, B, w, x))
        cps.append((MeshObjective(cc[0], cc[1], cc[2], m.n_nodes), cc[3], torch.empty_like(cc[3])))
    torch.cuda.synchronize()
    ms_g = _rotating(lambda i: cps[i][0].gradient(cps[i][1], out=cps[i][2]), len(cps),
                     args.steps, args.warmup)
    ms_f = _rotating(lambda i: cps[i][0].objective(cps[i][1]), len(cps), args.steps, args.warmup)
    for o, *_ in cps:
        o.timing(1)
    for i in range(args.steps):
        cps[i % len(cps)][0].gradient(cps[i % len(cps)][1], out=cps[i % len(cps)][2])
    torch.cuda.synchronize()
    kms, kn = 0.0, 0
    for o, *_ in cps:
        a, b = o.timing_read()
        o.timing(0)
        kms, kn = kms + a, kn + b
    kms /= max(kn, 1)
    f, g = cps[0][0].gradient(cps[0][1])
    gh = g.cpu().numpy().astype(np.float64)
    m32 = m.astype(np.float32)
    f_r, g_r = oracle.mesh_gradient(m.n_nodes, m.conn, m32.B.astype(np.float64),
                                    m32.w.astype(np.float64), m32.x.astype(np.float64))
    f_64, g_64 = oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    gb = algorithmic_bytes(m.n_nodes, m.n_elems, 8, 4, True) / 1e9
    return {"gradient_ms": round(ms_g, 5), "objective_ms": round(ms_f, 5),
            "GBps": round(gb / (ms_g * 1e-3), 2), "pct_hbm_peak": round(100 * gb / (ms_g * 1e-3) / PEAK_HBM_GBS, 2),
            "gradient_over_objective": round(ms_g / ms_f, 4),
            "kernel_ms": round(kms, 5), "kernel_GBps": round(gb / (kms * 1e-3), 2),
            "algorithmic_bytes": int(gb * 1e9),
            "error_vs_rounded_input_oracle": {"f": abs(f.item() - f_r) / abs(f_r), "grad": rel(gh, g_r)},
            "error_vs_fp64_input_oracle": {"f": abs(f.item() - f_64) / abs(f_64), "grad": rel(gh, g_64)},
            "cache": f"cold ({len(cps)} rotating copies)"}


def _batch_vs_per_instance(args):
    """256 uneven hex meshes: the one-launch batched gradient against 256
    per-instance gradient calls on the same GPU, same inputs."""
    import torch
    from paper_2507_13204_amd import MeshBatch, MeshObjective, inputs
    bt = inputs.uneven_batch(args.batch_n)
    dev = torch.device("cuda:0")
    conn = torch.from_numpy(bt.conn).to(dev)
    B = torch.from_numpy(bt.B).to(dev)
    w = torch.from_numpy(bt.w).to(dev)
    x = torch.from_numpy(bt.x).to(dev)
    N, E = int(bt.x.shape[0]), int(bt.conn.shape[0])
    gbytes = algorithmic_bytes(N, E, 8, 8, True) / 1e9
    g = torch.empty_like(x)
    f = torch.empty(bt.n_inst, dtype=torch.float64, device=dev)
    ob = MeshBatch(bt.inst, conn, B, w)
    ms_b = _timed(lambda: ob.gradient(x, out=g, f_out=f), args.steps, args.warmup)
    k_ms = _hook_ms(ob, lambda: ob.gradient(x, out=g, f_out=f), args.steps)
    ob.close()
    plans = []
    for i in range(bt.n_inst):
        nn, ne, no, eo = (int(v) for v in bt.inst[i])
        plans.append((MeshObjective(conn[eo:eo + ne], B[eo:eo + ne], w[eo:eo + ne], nn),
                      x[no:no + nn], g[no:no + nn], f[i:i + 1].view(())))

    def per_instance():
        for p, xi, gi, fi in plans:
            p.gradient(xi, out=gi, f_out=fi)

    ms_pi = _timed(per_instance, max(3, args.steps // 4), 1)
    for p, *_ in plans:
        p.close()
    return {"workload": f"{bt.n_inst} hex meshes, sides log-uniform in [10,100], {N} nodes, "
                        f"{E} elements, FP64 gradient, atomic adjoint",
            "batched_ms": round(ms_b, 4), "batched_instances_per_s": round(bt.n_inst / (ms_b * 1e-3), 1),
            "batched_GBps": round(gbytes / (ms_b * 1e-3), 2),
            "batched_kernel_ms": round(k_ms, 4),
            "batched_kernel_frac_hbm_peak": round(gbytes / (k_ms * 1e-3) / PEAK_HBM_GBS, 4),
            "per_instance_ms": round(ms_pi, 4),
            "per_instance_instances_per_s": round(bt.n_inst / (ms_pi * 1e-3), 1),
            "per_instance_GBps": round(gbytes / (ms_pi * 1e-3), 2),
            "batched_over_per_instance_speedup": round(ms_pi / ms_b, 3),
            "algorithmic_bytes": int(gbytes * 1e9)}


def _other_configs(args):
    """The dense row reduction (10^4 x 10^4, FP64) and the batched dense
    products (4096^2 by 4096 x 1024, FP64 and FP32 matrix cores) in the hex
    line: times per call, the dominant kernel from the event hook against its
    roofline, and the gradient / objective ratios."""
    import torch
    from paper_2507_13204_amd import BatchedDense, DenseObjective, inputs
    dev = torch.device("cuda:0")
    steps, warm = 10, 3
    res = {}
    n = args.dense_n
    d = inputs.dense(n)
    A = torch.from_numpy(d.A).to(dev)
    w = torch.from_numpy(d.w).to(dev)
    x = torch.from_numpy(d.x).to(dev)
    obj = DenseObjective(A, w)
    g = torch.empty_like(x)
    ms_g = _timed(lambda: obj.gradient(x, out=g), steps, warm)
    ms_f = _timed(lambda: obj.objective(x), steps, warm)
    k_g = _hook_ms(obj, lambda: obj.gradient(x, out=g), steps)
    gbytes = (n * n + 3 * n) * 8 / 1e9
    res["dense"] = {"workload": f"dense {n}x{n} f64, one pass over A for f and the gradient",
                    "gradient_ms": round(ms_g, 5), "objective_ms": round(ms_f, 5),
                    "gradient_over_objective": round(ms_g / ms_f, 4),
                    "GBps": round(gbytes / (ms_g * 1e-3), 2),
                    "kernel": "k_dense_fused", "kernel_ms": round(k_g, 5),
                    "kernel_frac_hbm_peak": round(gbytes / (k_g * 1e-3) / PEAK_HBM_GBS, 4)}
    obj.close()
    del A, w, x, g, d
    torch.cuda.empty_cache()
    m_, n_ = args.bd_m, args.bd_n
    b = inputs.batched_dense(m_, n_)
    flop = 2.0 * m_ * m_ * n_
    for dt, tdt, peak in (("f64", torch.float64, 78.6), ("f32", torch.float32, 157.3)):
        A = torch.from_numpy(b.A).to(dev, tdt)
        W = torch.from_numpy(b.W).to(dev, tdt)
        X = torch.from_numpy(b.X).to(dev, tdt)
        o = BatchedDense(A, W, ckpt="store")
        G = torch.empty_like(X)
        fbar = torch.ones(1, dtype=torch.float64, device=dev)
        ms_f = _timed(lambda: o.objective(X), steps, warm)
        ms_b = _timed(lambda: o.adjoint(X, fbar, out=G), steps, warm)
        ms_g = _timed(lambda: o.gradient(X, out=G), steps, warm)
        k_f = _hook_ms(o, lambda: o.objective(X), steps)
        res[f"bdense_{dt}"] = {
            "workload": f"batched dense A {m_}x{m_}, X {m_}x{n_}, {dt} matrix cores"
                        + (", each 16-deep k-tile added into FP64" if dt == "f32" else ""),
            "forward_kernel_ms": round(k_f, 5),
            "forward_TFLOPs": round(flop / (k_f * 1e-3) / 1e12, 3),
            "forward_frac_peak": round(flop / (k_f * 1e-3) / 1e12 / peak, 4),
            "peak_TFLOPs": peak, "gradient_ms": round(ms_g, 5),
            "fwd_plus_bwd_over_fwd": round((ms_f + ms_b) / ms_f, 4)}
        o.close()
        del A, W, X, G
        torch.cuda.empty_cache()
    return res


def _small_sweeps(args):
    """The launch-bound cases on a coarse grid of sizes: the 1D chain through
    the mesh path and the paper's own example (gather schedule, gradients in
    x and b), gradient / objective wall-clock ratios per size."""
    import numpy as np
    import torch
    from paper_2507_13204_amd import Laplace1D, MeshObjective, inputs
    dev = torch.device("cuda:0")
    steps, warm = 20, 5
    sizes = [1, 100, 1000, 2000, 4000, 6000, 8000, 10_000]
    chain, paper = [], []
    for n in sizes:
        if n >= 2:
            m = inputs.chain(n)
            obj = MeshObjective(torch.from_numpy(m.conn).to(dev), torch.from_numpy(m.B).to(dev),
                                torch.from_numpy(m.w).to(dev), n)
            x = torch.from_numpy(m.x).to(dev)
            g = torch.empty_like(x)
            f = torch.empty((), dtype=torch.float64, device=dev)
            ms_g = _timed(lambda: obj.gradient(x, out=g, f_out=f), steps, warm)
            ms_f = _timed(lambda: obj.objective(x, f_out=f), steps, warm)
            chain.append((n, round(ms_f * 1e3, 3), round(ms_g * 1e3, 3), round(ms_g / ms_f, 4)))
            obj.close()
        rng = np.random.default_rng(n)
        x = torch.from_numpy(rng.uniform(-1, 1, n)).to(dev)
        b = torch.from_numpy(rng.uniform(-1, 1, n)).to(dev)
        lp = Laplace1D(n)
        gx, gb = torch.empty_like(x), torch.empty_like(b)
        f = torch.empty((), dtype=torch.float64, device=dev)
        ms_g = _timed(lambda: lp.gradient(x, b, gx=gx, gb=gb, f_out=f), steps, warm)
        ms_f = _timed(lambda: lp.objective(x, b, f_out=f), steps, warm)
        paper.append((n, round(ms_f * 1e3, 3), round(ms_g * 1e3, 3), round(ms_g / ms_f, 4)))
        lp.close()
    return {"chain": {"workload": "1D chain through the mesh path, n nodes",
                      "n_us_f_us_grad_ratio": chain,
                      "max_ratio": max(r[3] for r in chain)},
            "paper_example": {"workload": "the paper's ||A(3x) - b||^2, dim(x) = n, gradients in x and b",
                              "n_us_f_us_grad_ratio": paper,
                              "max_ratio": max(r[3] for r in paper),
                              "paper_us_f_grad": PAPER_US}}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def _hook_ms(plan, fn, steps):
    import torch
    plan.timing(1)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms, n = plan.timing_read()
    plan.timing(0)
    return ms / max(n, 1)


def _line(metric, value, unit, args, ms, dtype, config, higher=True, **extra):
    out = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
           "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded)", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_dense(args):
    """A 10,000 x 10,000 FP64 row reduction: f and its gradient in one pass over A."""
    import numpy as np
    import torch
    import oracle
    from paper_2507_13204_amd import DenseObjective, inputs
    n = args.dense_n
    d = inputs.dense(n)
    dev = torch.device("cuda:0")
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    esz = 8 if args.dtype == "f64" else 4
    A = torch.from_numpy(d.A).to(dev, tdt)
    w = torch.from_numpy(d.w).to(dev, tdt)
    x = torch.from_numpy(d.x).to(dev, tdt)
    obj = DenseObjective(A, w)
    g = torch.empty_like(x)
    ms_g = _timed(lambda: obj.gradient(x, out=g), args.steps, args.warmup)
    ms_f = _timed(lambda: obj.objective(x), args.steps, args.warmup)
    k_g = _hook_ms(obj, lambda: obj.gradient(x, out=g), args.steps)
    gbytes = (n * n + 3 * n) * esz / 1e9
    t0 = time.perf_counter()
    oracle.dense_gradient(d.A, d.x, d.w)
    cpu_s = time.perf_counter() - t0
    _line("dense row-reduction gradient GB/s (A n x n, one pass over A)", gbytes / (ms_g * 1e-3),
          "GB/s", args, ms_g, args.dtype,
          {"workload": f"dense {n}x{n} {args.dtype}, one workgroup team per row band"},
          gradient_over_objective=round(ms_g / ms_f, 4), objective_ms=round(ms_f, 5),
          roofline={"bound": "hbm", "achieved": round(gbytes / (k_g * 1e-3), 2),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(gbytes / (k_g * 1e-3) / PEAK_HBM_GBS, 4), "traffic": None,
                    "kernel": "k_dense_fused", "kernel_ms": round(k_g, 5)},
          cpu_baseline={"value": round(gbytes / cpu_s, 3), "unit": "GB/s", "cores": 1,
                        "kind": "oracle", "sample": f"one Dot2 FP64 gradient, {n}x{n}"})


def bench_bdense(args):
    """A 4096^2, X 4096 x 1024: forward product with the psi epilogue and the
    backward product A^T V on the matrix cores."""
    import numpy as np
    import torch
    from paper_2507_13204_amd import BatchedDense, inputs
    m, n = args.bd_m, args.bd_n
    b = inputs.batched_dense(m, n)
    dev = torch.device("cuda:0")
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    A = torch.from_numpy(b.A).to(dev, tdt)
    W = torch.from_numpy(b.W).to(dev, tdt)
    X = torch.from_numpy(b.X).to(dev, tdt)
    res = {}
    for ckpt in ("store", "recompute"):
        obj = BatchedDense(A, W, ckpt=ckpt)
        G = torch.empty_like(X)
        fbar = torch.ones(1, dtype=torch.float64, device=dev)
        ms_f = _timed(lambda: obj.objective(X), args.steps, args.warmup)
        ms_b = _timed(lambda: obj.adjoint(X, fbar, out=G), args.steps, args.warmup)
        ms_g = _timed(lambda: obj.gradient(X, out=G), args.steps, args.warmup)
        k_f = _hook_ms(obj, lambda: obj.objective(X), args.steps)
        res[ckpt] = {"objective_ms": round(ms_f, 4), "adjoint_ms": round(ms_b, 4),
                     "gradient_ms": round(ms_g, 4), "fwd_kernel_ms": round(k_f, 4),
                     "fwd_plus_bwd_over_fwd": round((ms_f + ms_b) / ms_f, 4)}
        obj.close()
    flop = 2.0 * m * m * n
    peak = 78.6 if args.dtype == "f64" else 157.3
    kf = res["store"]["fwd_kernel_ms"]
    Xs = np.ascontiguousarray(b.X[:, :64])
    t0 = time.perf_counter()
    _ = b.A @ Xs
    cpu_s = time.perf_counter() - t0
    _line("batched dense gradient TFLOP/s (A m x m, X m x n, MFMA)",
          2 * flop / (res["store"]["gradient_ms"] * 1e-3) / 1e12, "TFLOP/s", args,
          res["store"]["gradient_ms"], args.dtype,
          {"workload": f"batched dense A {m}x{m}, X {m}x{n}, {args.dtype} MFMA"},
          variants=res,
          roofline={"bound": "mfma", "achieved": round(flop / (kf * 1e-3) / 1e12, 3),
                    "peak": peak, "unit": "TFLOP/s",
                    "frac": round(flop / (kf * 1e-3) / 1e12 / peak, 4), "traffic": None,
                    "kernel": "k_gemm_mfma forward (psi epilogue)", "kernel_ms": kf},
          cpu_baseline={"value": round(2 * m * m * 64 / cpu_s / 1e12, 5), "unit": "TFLOP/s",
                        "cores": os.cpu_count(), "kind": "oracle",
                        "sample": "the oracle's NumPy FP64 product A @ X on 64 columns"})


def bench_batch(args):
    """256 uneven hex meshes: one launch over all instances' tiles (eager and HIP-graph replay)
    against 256 per-instance gradient calls."""
    import numpy as np
    import torch
    from paper_2507_13204_amd import MeshBatch, MeshObjective, inputs
    from paper_2507_13204_amd import autotune
    bt = inputs.uneven_batch(args.batch_n)
    dev = torch.device("cuda:0")
    conn = torch.from_numpy(bt.conn).to(dev)
    B = torch.from_numpy(bt.B).to(dev)
    w = torch.from_numpy(bt.w).to(dev)
    x = torch.from_numpy(bt.x).to(dev)
    N, E = int(bt.x.shape[0]), int(bt.conn.shape[0])
    gbytes = (E * 8 * 4 + E * 8 * 8 + E * 8 + 2 * N * 8) / 1e9
    tuned = autotune.tune_batch(bt.inst, conn, B, w, x, use_cache=False)
    res = {"autotune": tuned}
    g = torch.empty_like(x)
    f = torch.empty(bt.n_inst, dtype=torch.float64, device=dev)
    for ckpt in ("recompute", "store"):
        ob = MeshBatch(bt.inst, conn, B, w, ckpt=ckpt, block=tuned["block"], tile=tuned["tile"])
        ms_g = _timed(lambda: ob.gradient(x, out=g, f_out=f), args.steps, args.warmup)
        fbar = torch.ones(bt.n_inst, dtype=torch.float64, device=dev)
        ms_fb = _timed(lambda: (ob.objective(x, f_out=f), ob.adjoint(x, fbar, out=g)),
                       args.steps, args.warmup)
        res[ckpt] = {"gradient_ms": round(ms_g, 4), "objective_plus_adjoint_ms": round(ms_fb, 4)}
        if ckpt == "recompute":
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(s):
                ob.gradient(x, out=g, f_out=f, stream=s)
                with torch.cuda.graph(graph, stream=s):
                    ob.gradient(x, out=g, f_out=f, stream=s)
            torch.cuda.current_stream().wait_stream(s)
            ms_graph = _timed(graph.replay, args.steps, args.warmup)
            res["graph_gradient_ms"] = round(ms_graph, 4)
            k_ms = _hook_ms(ob, lambda: ob.gradient(x, out=g, f_out=f), args.steps)
        ob.close()
    # per-instance form: one plan per mesh, one gradient call each
    plans = []
    for i in range(bt.n_inst):
        nn, ne, no, eo = (int(v) for v in bt.inst[i])
        plans.append((MeshObjective(conn[eo:eo + ne], B[eo:eo + ne], w[eo:eo + ne], nn),
                      x[no:no + nn], g[no:no + nn], f[i:i + 1].view(())))

    def per_instance():
        for p, xi, gi, fi in plans:
            p.gradient(xi, out=gi, f_out=fi)

    ms_pi = _timed(per_instance, max(3, args.steps // 10), 1)
    res["per_instance_ms"] = round(ms_pi, 4)
    best = min(res["recompute"]["gradient_ms"], res["graph_gradient_ms"])
    _line("uneven batch gradient throughput (instances/s), 256 hex meshes in one launch",
          bt.n_inst / (best * 1e-3), "instances/s", args, best, "f64",
          {"workload": f"{bt.n_inst} hex meshes, sides log-uniform in [10,100], "
                       f"{N} nodes, {E} elements"},
          GBps=round(gbytes / (best * 1e-3), 2),
          per_instance_instances_per_s=round(bt.n_inst / (ms_pi * 1e-3), 2),
          batched_over_per_instance_speedup=round(ms_pi / best, 3),
          variants=res,
          roofline={"bound": "hbm", "achieved": round(gbytes / (k_ms * 1e-3), 2),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(gbytes / (k_ms * 1e-3) / PEAK_HBM_GBS, 4), "traffic": None,
                    "kernel": "k_batch_tiles (gradient, atomic)", "kernel_ms": round(k_ms, 5)},
          cpu_baseline=_batch_cpu(bt, args.cpu_seconds))


def _batch_cpu(bt, budget_s):
    """The oracle on whole instances of the batch, in work-list order, until
    the budget is spent; instances per second."""
    import oracle
    order = sorted(range(bt.n_inst), key=lambda i: -int(bt.inst[i][1]))
    t0 = time.perf_counter()
    done = 0
    for i in order[::max(1, bt.n_inst // 32)]:
        m = bt.instance(i)
        oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    frac = sum(int(bt.inst[i][1]) for i in order[::max(1, bt.n_inst // 32)][:done]) / max(
        1, int(bt.inst[:, 1].sum()))
    return {"value": round(frac * bt.n_inst / el, 3), "unit": "instances/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{done} instances (every {max(1, bt.n_inst // 32)}th of the size-ordered list, "
                      f"{100 * frac:.1f}% of the elements) in {el:.1f} s, scaled to the batch"}


def bench_chain(args):
    """The 1D chain over the paper's sweep of dim(x) = 1, 100, ..., 10,000."""
    import torch
    from paper_2507_13204_amd import MeshObjective, inputs
    dev = torch.device("cuda:0")
    sweep = []
    for n in [1] + list(range(100, 10001, 100)):
        m = inputs.chain(n)
        if m.n_elems == 0:
            continue
        obj = MeshObjective(torch.from_numpy(m.conn).to(dev), torch.from_numpy(m.B).to(dev),
                            torch.from_numpy(m.w).to(dev), n)
        x = torch.from_numpy(m.x).to(dev)
        g = torch.empty_like(x)
        f = torch.empty((), dtype=torch.float64, device=dev)
        ms_g = _timed(lambda: obj.gradient(x, out=g, f_out=f), args.steps, args.warmup)
        ms_f = _timed(lambda: obj.objective(x, f_out=f), args.steps, args.warmup)
        sweep.append((n, round(ms_f * 1e3, 3), round(ms_g * 1e3, 3), round(ms_g / ms_f, 4)))
        obj.close()
    ratios = sorted(r[3] for r in sweep)
    import oracle
    m = inputs.chain(10_000)
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 1.0:
        oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
        reps += 1
    cpu_us = (time.perf_counter() - t0) / reps * 1e6
    nbytes = m.conn.nbytes + m.B.nbytes + m.w.nbytes + 2 * m.x.nbytes
    _line("1D chain gradient/objective wall-clock ratio (max over n = 100..10,000)", ratios[-1],
          "ratio", args, sweep[-1][2] / 1e3, "f64",
          {"workload": "1D chain, n = 100..10,000 (the paper's sweep of dim(x))"}, higher=False,
          median_ratio=ratios[len(ratios) // 2], sweep_n_us_f_us_grad_ratio=sweep,
          roofline={"bound": "hbm", "achieved": round(nbytes / (sweep[-1][2] * 1e-6) / 1e9, 3),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(nbytes / (sweep[-1][2] * 1e-6) / 1e9 / PEAK_HBM_GBS, 6),
                    "traffic": None, "kernel": "whole gradient call at n = 10,000 (launch-bound)"},
          cpu_baseline={"value": round(cpu_us, 2), "unit": "us per gradient (n = 10,000)",
                        "cores": 1, "kind": "oracle", "sample": f"{reps} oracle gradients"})


# The paper's wall-clock times of f and of its generated gradient for dim(x) = 1
# and 10,000 (figures of the results section), microseconds.
PAPER_US = {"H100": {1: (41.79, 74.70), 10000: (47.82, 85.44)},
            "MI250X (one GCD)": {1: (89.67, 194.68), 10000: (113.62, 233.82)},
            "Ponte Vecchio": {1: (28.16, 56.07), 10000: (38.11, 68.24)}}


def _paper_cpu():
    import numpy as np
    import oracle
    rng = np.random.default_rng(10000)
    x, b = rng.uniform(-1, 1, 10000), rng.uniform(-1, 1, 10000)
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 1.0:
        oracle.laplace1d_gradient(x, b)
        reps += 1
    us = (time.perf_counter() - t0) / reps * 1e6
    return {"value": round(us, 2), "unit": "us per gradient (n = 10,000)", "cores": 1,
            "kind": "oracle", "sample": f"{reps} oracle gradients in x and b"}


def bench_paper(args):
    """The paper's own example, f(x, b) = ||A(3x) - b||^2, swept over
    dim(x) = 1, 100, ..., 10,000 as in its results section; gradient in x and b."""
    import numpy as np
    import torch
    from paper_2507_13204_amd import Laplace1D
    dev = torch.device("cuda:0")
    res = {}
    for adj in ("gather", "atomic"):
        sweep = []
        for n in [1] + list(range(100, 10001, 100)):
            rng = np.random.default_rng(n)
            x = torch.from_numpy(rng.uniform(-1, 1, n)).to(dev)
            b = torch.from_numpy(rng.uniform(-1, 1, n)).to(dev)
            lp = Laplace1D(n, adjoint=adj)
            gx, gb = torch.empty_like(x), torch.empty_like(b)
            f = torch.empty((), dtype=torch.float64, device=dev)
            ms_g = _timed(lambda: lp.gradient(x, b, gx=gx, gb=gb, f_out=f), args.steps, args.warmup)
            ms_f = _timed(lambda: lp.objective(x, b, f_out=f), args.steps, args.warmup)
            sweep.append((n, round(ms_f * 1e3, 3), round(ms_g * 1e3, 3), round(ms_g / ms_f, 4)))
            lp.close()
        res[adj] = sweep
    r = sorted(v[3] for v in res["gather"])
    _line("paper example ||A(3x)-b||^2: gradient/objective wall-clock ratio, max over "
          "dim(x) = 1..10,000", r[-1], "ratio", args, res["gather"][-1][2] / 1e3, "f64",
          {"workload": "the paper's section 4 example, 1D Laplacian, dim(x) = 1, 100, ..., 10,000"},
          higher=False, median_ratio=r[len(r) // 2],
          atomic_schedule_max_ratio=max(v[3] for v in res["atomic"]),
          paper_us_f_grad=PAPER_US, sweep_gather=res["gather"], sweep_atomic=res["atomic"],
          roofline={"bound": "hbm", "achieved": round(32 * 10000 / (res["gather"][-1][2] * 1e-6) / 1e9, 3),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(32 * 10000 / (res["gather"][-1][2] * 1e-6) / 1e9 / PEAK_HBM_GBS, 6),
                    "traffic": None, "kernel": "whole gradient call at n = 10,000 (launch-bound)"},
          cpu_baseline=_paper_cpu())


def _program_cpu(budget_s: float = 5.0):
    """The program oracle (forward Jacobian accumulation) on hex meshes of
    growing side until the budget is spent; rate in algorithmic GB/s."""
    from oracle import program as OP
    from paper_2507_13204_amd import inputs
    m = inputs.hex_mesh(64, seed=1)
    case = inputs.program_mesh(m)
    done_bytes, t0, runs = 0, time.perf_counter(), 0
    while time.perf_counter() - t0 < budget_s:
        OP.gradient(case.spec, case.inputs)
        done_bytes += algorithmic_bytes(m.n_nodes, m.n_elems, 8, 8, True)
        runs += 1
    dt = time.perf_counter() - t0
    return {"value": round(done_bytes / dt / 1e9, 5), "unit": "GB/s (algorithmic)", "cores": 1,
            "kind": "oracle", "sample": f"{runs} program-oracle gradients of the 64^3 hex mesh "
            "(forward Jacobians in scipy.sparse)"}


def bench_program(args):
    """Composed programs (pg_prog_*): the 128^3 hex objective written as
    constructs (gather, map psi, weight, sum) against the fused element
    kernel, and the paper's example at dim(x) = 10,000 against its hand-fused
    form.  The difference is what fusing the constructs buys."""
    import torch
    from paper_2507_13204_amd import Laplace1D, MeshObjective, Program, inputs
    dev = torch.device("cuda:0")
    m = inputs.hex_mesh(args.side)
    case = inputs.program_mesh(m)
    prog = Program.from_spec(case.spec, device=dev).plan(dev)
    x = torch.from_numpy(m.x).to(dev)
    f = torch.empty((), dtype=torch.float64, device=dev)
    g = [torch.empty_like(x)]
    ms_prog = _timed(lambda: prog.run([x], grads=g, f_out=f), args.steps, args.warmup)
    ms_prog_f = _timed(lambda: prog.run([x], grads=None, f_out=f), args.steps, args.warmup)
    info = prog.info()
    del prog
    prog0 = Program.from_spec(case.spec, device=dev, fusion=0).plan(dev)
    ms_unfused = _timed(lambda: prog0.run([x], grads=g, f_out=f), args.steps, args.warmup)
    del prog0
    mo = MeshObjective(torch.from_numpy(m.conn).to(dev), torch.from_numpy(m.B).to(dev),
                       torch.from_numpy(m.w).to(dev), m.n_nodes)
    gf = torch.empty_like(x)
    ms_fused = _timed(lambda: mo.gradient(x, out=gf, f_out=f), args.steps, args.warmup)
    mo.close()
    pc = inputs.program_paper(10000, seed=10000)
    pp = Program.from_spec(pc.spec, device=dev).plan(dev)
    xs = [torch.from_numpy(v).to(dev) for v in pc.inputs]
    gp = [torch.empty_like(v) for v in xs]
    ms_pp = _timed(lambda: pp.run(xs, grads=gp, f_out=f), args.steps, args.warmup)
    lp = Laplace1D(10000)
    ms_lp = _timed(lambda: lp.gradient(xs[0], xs[1], gx=gp[0], gb=gp[1], f_out=f), args.steps,
                   args.warmup)
    lp.close()
    alg = algorithmic_bytes(m.n_nodes, m.n_elems, 8, 8, True)
    gbs = alg / (ms_prog * 1e-3) / 1e9
    _line(f"composed-program gradient throughput, {args.side}^3 hex mesh (algorithmic bytes)",
          gbs, "GB/s", args, ms_prog, "f64",
          {"workload": f"hex mesh {args.side}^3 nodes as constructs gather -> map psi -> "
                       "weight -> sum, FP64, reverse pass generated construct by construct"},
          program_objective_ms=round(ms_prog_f, 5), fused_gradient_ms=round(ms_fused, 5),
          program_unfused_ms=round(ms_unfused, 5),
          program_over_fused=round(ms_prog / ms_fused, 3), program_info=info,
          paper_example_program_us=round(ms_pp * 1e3, 2),
          paper_example_fused_us=round(ms_lp * 1e3, 2),
          roofline={"bound": "hbm", "achieved": round(gbs, 3), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 6), "traffic": None,
                    "kernel": "whole program gradient call (fused groups)"},
          cpu_baseline=None if args.no_cpu else _program_cpu())


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    {"hex": bench_hex, "dense": bench_dense, "bdense": bench_bdense, "batch": bench_batch,
     "chain": bench_chain, "paper": bench_paper, "program": bench_program}[args.workload](args)
    if args.calibrate_copy:
        # a plain 512 MiB device copy: the scale for rocprofv3's byte counters
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
