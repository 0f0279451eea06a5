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
    ap.add_argument("--adjoint", default="atomic", choices=["atomic", "gather", "colour"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--copies", type=int, default=3, help="rotating input copies")
    ap.add_argument("--scatter", type=int, default=0, help="0 combine in LDS, 1 direct atomics")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=6.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 512 MiB device copy (scale for byte counters)")
    return ap.parse_args()


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


def cpu_baseline(m, budget_s: float, gbytes: float):
    import numpy as np
    import oracle
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        oracle.mesh_gradient(m.n_nodes, m.conn, m.B, m.w, m.x)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end and len(times) >= 3:
            break
    med = float(np.median(times))
    return {"value": round(gbytes / med, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"full {m.name} FP64 gradient (f and grad), single-threaded C oracle, "
                      f"median of {len(times)} runs = {med * 1e3:.1f} ms",
            "cpu": platform.processor() or platform.machine()}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_13204_amd import MeshObjective, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
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
                     "kernel": f"k_mesh_elem (gradient, {args.adjoint})",
                     "kernel_ms": round(kms_grad, 5),
                     "algorithmic_bytes": int(gbytes * 1e9)},
    }

    if not args.no_variants:
        variants = {}
        for adj in ("atomic", "gather", "colour"):
            if adj == args.adjoint:
                continue
            o2 = MeshObjective(conn, B, w, m.n_nodes, adjoint=adj)
            g2 = torch.empty_like(x)
            for _ in range(3):
                o2.gradient(x, out=g2)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                o2.gradient(x, out=g2)
            e1.record()
            torch.cuda.synchronize()
            vms = e0.elapsed_time(e1) / 20
            variants[adj] = {"ms": round(vms, 5), "GBps_algorithmic": round(gbytes / (vms * 1e-3), 2),
                             "over_objective": round(vms / ms_obj, 4), "cache": "warm"}
            o2.close()
        out["variants"] = variants

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_seconds, gbytes)

    if args.calibrate_copy:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
