"""Throughput of the coupled LB freezing step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32]

Workload: the 2D droplet freezing case scaled to a 2048 x 2048 grid (drop
radius 512 on the cold wall, interface width 4, D2Q9 flow + D2Q5 phase
field, enthalpy and solute), synthetic seeded initial fields, inputs resident
in HBM when timing starts.  One step = one launch of the fused step kernel =
one pass of the whole method over the grid.  Prints one JSON line.

The roofline entry uses the algorithmic bytes of one node update (every
population read once and written once, plus the previous-time-level fields
the scheme carries: 24 populations and 6 scalars, 240 B in FP32) divided by
the average launch time measured with HIP events on the solver's stream.
The CPU baseline is the FP64 oracle on the host cores, timed on whole steps of
the same 2048 x 2048 workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
POP_BYTES = {"f32": 4, "f16": 2, "bf16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step2d_2048.json")
# sources of the timed kernel: the stored counter figures hold only while
# these are unchanged
KERNEL_SOURCES = ("paper_2511_09422_amd/csrc/lbfz_2d.hip",
                  "paper_2511_09422_amd/csrc/lbfz_common.hpp",
                  "paper_2511_09422_amd/csrc/lbfz_kernels.hpp")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def bytes_per_node(storage: str) -> int:
    # 24 populations read + written, 6 FP32 scalars (f_s, p, u_x, u_y, phi, C)
    # read + written
    return 2 * 24 * POP_BYTES[storage] + 2 * 6 * 4


def cpu_baseline(cfg, phi, T, C, budget_s: float = 12.0) -> dict:
    from oracle.lbref import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    o = Oracle(cfg, phi, T, C, threads=threads)
    o.step(1)                      # first touch of the oracle's arrays
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 20:
            break
    dt = time.perf_counter() - t0
    N = cfg["nx"] * cfg["ny"]
    return {"value": round(N * n / dt / 1e6, 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} full steps of the {cfg['nx']}x{cfg['ny']} workload after one "
                      f"untimed step, FP64, OpenMP over nodes"}


def load_traffic(kernel_tag: str):
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_tag") != kernel_tag or d.get("source_sha256") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=sorted(POP_BYTES))
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2511_09422_amd.lbfz import Solver
    from paper_2511_09422_amd.workloads import droplet_2d

    n = args.n
    cfg, phi, T, C = droplet_2d(n, n, R=n / 4.0, seed=0)
    print(f"bench: 2D droplet {n}x{n}, storage {args.storage}, warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)
    solver = Solver(cfg, phi, T, C, device=0, storage=args.storage)
    stream = solver.stream
    solver.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    solver.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    tot = solver.totals()
    if tot["nonfinite"]:
        print("bench: non-finite state", file=sys.stderr)
        sys.exit(1)
    N = n * n
    ms_per_step = ms_total / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    bpn = bytes_per_node(args.storage)
    achieved = bpn * N / (ms_per_step * 1e-3) / 1e9
    tag = f"k_step2d_{args.storage}_{n}"
    traffic = load_traffic(tag)
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    out = {
        "metric": "coupled-field MLUPS (FP32 vs FP16-store); sweep cases/s; surrogate speedup",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D droplet freezing {n}x{n}, R={n // 4}, interface width 4, "
                               "D2Q9+3xD2Q5, FP32 arithmetic",
                   "grid": [n, n], "storage": args.storage, "bytes_per_node": bpn,
                   "wall_s": round(wall, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, phi, T, C)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
