"""Throughput of the coupled LB freezing step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32]

Workload: the 2D droplet freezing case scaled to a 2048 x 2048 grid (drop
radius 512 on the cold wall, interface width 4, D2Q9 flow + D2Q5 phase
field, enthalpy and solute), synthetic seeded initial fields, inputs resident
in HBM when timing starts.  One step = one launch of the fused step kernel =
one pass of the whole method over the grid.  The headline is FP32 storage;
the FP16 and BF16 storage forms and the 3D droplet (256^3 with its obstacle,
two launches per step) are timed the same way and reported in the same JSON
line.

The roofline entry uses the algorithmic bytes of one node update (every
population read once and written once, plus the previous-time-level fields
the scheme carries: 24 populations and 6 FP32 scalars, 240 B with FP32
storage, 144 B with 16-bit storage) divided by the average launch time
measured with HIP events on the solver's stream; the 16-bit forms also
report the fraction at the 172 B/node their design moves (FP32 rest
populations and the decode references).
The CPU baseline is the FP64 oracle on the host cores, timed on whole steps of
the same 2048 x 2048 workload.
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
POP_BYTES = {"f32": 4, "f16": 2, "bf16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# sources of the timed kernel: the stored counter figures hold only while
# these are unchanged
KERNEL_SOURCES = ("paper_2511_09422_amd/csrc/lbfz_2d.hip",
                  "paper_2511_09422_amd/csrc/lbfz_3d.hip",
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
    """Algorithmic bytes of one 2D node update: the 24 populations (D2Q9 + 3 x
    D2Q5) read and written once in the storage format, and the 6 FP32
    previous-level scalars (f_s, p, u_x, u_y, phi, C) read and written: 240 B
    with FP32 storage, 144 B with 16-bit storage."""
    return 2 * 24 * POP_BYTES[storage] + 2 * 6 * 4


def design_bytes_per_node(storage: str) -> int:
    """Bytes the 2D step is designed to move per node: the algorithmic bytes
    for FP32 storage; with 16-bit storage the rest populations stay FP32 (4 of
    the 24) and the decode references add scalars: 8 read (f_s, p, p two
    levels back, u_x, u_y, phi, C, T) and 7 written, 172 B."""
    if storage == "f32":
        return bytes_per_node(storage)
    return 2 * (4 * 4 + 20 * POP_BYTES[storage]) + (8 + 7) * 4


def bytes_per_node3d(storage: str) -> int:
    # the scheme's minimum: 40 populations (D3Q19 + 3 x D3Q7) read + written
    # and 8 FP32 previous-level scalars (f_s, p, u, phi, C, div u) read +
    # written; the two-launch design moves more (closure fields through HBM,
    # f, h, l read twice), which the measured traffic shows
    return 2 * 40 * POP_BYTES[storage] + 2 * 8 * 4


def cpu_baseline(cfg, phi, T, C, max_steps: int = 200, budget_s: float = 40.0) -> dict:
    """The FP64 oracle on the host cores: whole steps of the benchmark
    workload (up to max_steps, stopping once budget_s has passed) with OpenMP
    over nodes, two steps on one thread, and the 64^2 droplet's full
    1000-step run on all threads and on one."""
    from oracle.lbref import Oracle
    from paper_2511_09422_amd.workloads import droplet_2d
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    o = Oracle(cfg, phi, T, C, threads=threads)
    o.step(1)                      # first touch of the oracle's arrays
    t0 = time.perf_counter()
    n = 0
    while n < max_steps:
        o.step(1)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    del o
    N = cfg["nx"] * cfg["ny"]
    # the same oracle on one thread, two whole steps
    o1 = Oracle(cfg, phi, T, C, threads=1)
    o1.step(1)
    t1 = time.perf_counter()
    o1.step(2)
    dt1 = time.perf_counter() - t1
    del o1
    # the 64^2 droplet, 1000 steps from its initial fields
    c1, p1, T1, C1 = droplet_2d(64, 64, R=16.0, seed=0)
    small = {}
    for th in (threads, 1):
        o = Oracle(c1, p1, T1, C1, threads=th)
        t2 = time.perf_counter()
        o.step(1000)
        d2 = time.perf_counter() - t2
        del o
        small["threads_%d" % th] = {"s": round(d2, 3),
                                    "value": round(64 * 64 * 1000 / d2 / 1e6, 4)}
    return {"value": round(N * n / dt / 1e6, 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} full steps of the {cfg['nx']}x{cfg['ny']} workload after one "
                      f"untimed step ({dt:.1f} s), FP64, OpenMP over nodes",
            "single_thread": {"value": round(N * 2 / dt1 / 1e6, 4), "unit": "MLUPS",
                              "sample": "2 full steps after one untimed step"},
            "droplet_64": {"unit": "MLUPS", "sample": "the 64x64 droplet (R = 16), 1000 "
                                                      "steps from its initial fields",
                           **small},
            "cpu": cpu_model(), "nproc": os.cpu_count()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def load_traffic(kernel_tag: str):
    """Calibrated HBM bytes per launch of the tagged kernel from the stored
    counter summary, or None when it is missing or the kernel sources changed
    since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != kernel_source_hash():
        return None
    e = d.get("entries", {}).get(kernel_tag)
    return None if e is None else e.get("bytes_per_launch")


def time_form(cfg, phi, T, C, storage: str, warmup: int, steps: int, mask=None) -> dict:
    """Time `steps` steps of one storage form with HIP events on the solver's
    stream, after `warmup` untimed steps."""
    import torch
    from paper_2511_09422_amd.lbfz import Solver
    solver = Solver(cfg, phi, T, C, mask=mask, device=0, storage=storage)
    stream = solver.stream
    solver.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    solver.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / steps
    tot = solver.totals()
    solver.close()
    del solver
    torch.cuda.empty_cache()
    if tot["nonfinite"]:
        print(f"bench: non-finite state ({storage})", file=sys.stderr)
        sys.exit(1)
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    bpn = bytes_per_node(storage) if cfg["dim"] == 2 else bytes_per_node3d(storage)
    dbpn = design_bytes_per_node(storage) if cfg["dim"] == 2 else None
    achieved = bpn * N / (ms_per_step * 1e-3) / 1e9
    return {"ms_per_step": ms_per_step, "mlups": N / (ms_per_step * 1e-3) / 1e6,
            "bytes_per_node": bpn, "achieved": achieved, "wall": wall,
            "design_bytes_per_node": dbpn,
            "design_GBs": None if dbpn is None else dbpn * N / (ms_per_step * 1e-3) / 1e9}


def time_copy(nbytes: int, reps: int = 20) -> dict:
    """The library's streaming copy (lbfz_stream_copy) reading and writing
    nbytes in total (nbytes / 2 each way), timed with HIP events on its
    stream: the bandwidth this memory system gives a pure streaming kernel of
    the same volume as one step.  The runtime's device copy of the same
    buffers is timed beside it."""
    import torch
    from paper_2511_09422_amd.lbfz import lbfz_stream_copy
    n = (nbytes // 2) // 16 * 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()

    def run(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        for _ in range(reps):
            fn()
        ev1.record(st)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps
    ms = run(lambda: lbfz_stream_copy(b.data_ptr(), a.data_ptr(), 4 * n, st.cuda_stream))
    ms_rt = run(lambda: b.copy_(a))
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    if not ok:
        print("bench: the stream copy did not reproduce its source", file=sys.stderr)
        sys.exit(1)
    return {"bytes": 8 * n, "us": ms * 1e3, "GBs": 8 * n / (ms * 1e-3) / 1e9,
            "runtime_copy_us": ms_rt * 1e3, "runtime_copy_GBs": 8 * n / (ms_rt * 1e-3) / 1e9}


def time_pattern3d(m: int, reps: int = 10) -> dict:
    """The 3D FP32 step's memory pattern without its arithmetic, launch by
    launch (lbfz_stream_planes3d on an m^3 grid: the closure launch's 22
    planes in and 5 out, the collision launch's 50 in and 42 out, the
    populations pushed to their D3Q19 targets), timed with HIP events on its
    stream: what the two launches' access pattern can reach."""
    import torch
    from paper_2511_09422_amd.lbfz import lbfz_stream_planes3d
    N = m * m * m
    ps = (N + 63) // 64 * 64 + 1088
    a = torch.ones(50 * ps, dtype=torch.float32, device="cuda")
    b = torch.zeros(42 * ps, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    out = {}
    for name, (nr, nw) in (("closure", (22, 5)), ("collision", (50, 42))):
        fn = lambda: lbfz_stream_planes3d(b.data_ptr(), a.data_ptr(), m, m, m, ps, nr, nw,
                                          st.cuda_stream)
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        for _ in range(reps):
            fn()
        ev1.record(st)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        nbytes = (nr + nw) * 4 * N
        out[name] = {"planes_in": nr, "planes_out": nw, "bytes": nbytes, "us": round(ms * 1e3, 2),
                     "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    ok = bool(torch.equal(b[:N], a[:N]))
    del a, b
    torch.cuda.empty_cache()
    if not ok:
        print("bench: the 3D plane pattern did not move its source", file=sys.stderr)
        sys.exit(1)
    us = out["closure"]["us"] + out["collision"]["us"]
    nbytes = out["closure"]["bytes"] + out["collision"]["bytes"]
    out.update({"us": round(us, 2), "bytes_per_node": nbytes // N,
                "GB/s": round(nbytes / (us * 1e-6) / 1e9, 1),
                "frac_of_peak": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
    return out


def time_pattern(n: int, reps: int = 20) -> dict:
    """The step's own memory pattern without its arithmetic (lbfz_stream_planes:
    30 FP32 planes of an n x n grid read at each node and written to the rows
    the step's pushes land on), timed with HIP events on its stream: the
    bandwidth this access pattern can reach."""
    import torch
    from paper_2511_09422_amd.lbfz import lbfz_stream_planes
    N = n * n
    ps = (N + 63) // 64 * 64 + 1088
    a = torch.ones(30 * ps, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    st = torch.cuda.current_stream()
    fn = lambda: lbfz_stream_planes(b.data_ptr(), a.data_ptr(), n, n, ps, st.cuda_stream)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for _ in range(reps):
        fn()
    ev1.record(st)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    ok = bool(torch.equal(b[:N], a[:N]))
    del a, b
    torch.cuda.empty_cache()
    if not ok:
        print("bench: the plane pattern did not move its source", file=sys.stderr)
        sys.exit(1)
    nbytes = 2 * 30 * 4 * N
    return {"bytes": nbytes, "us": ms * 1e3, "GBs": nbytes / (ms * 1e-3) / 1e9}


def time_sweep(ncases: int, steps: int, case_steps: int, storage: str) -> dict:
    """The batched parameter sweep: ncases grids drawn by sweep_case(k), tuned,
    then whole cases -- `steps` batched steps (case_steps by default) --
    timed with HIP events (graph replays, one kernel node per step), and a
    few steps of the same grids with plain one-grid-at-a-time launches."""
    import torch
    from paper_2511_09422_amd.lbfz import Batch
    from paper_2511_09422_amd.workloads import sweep_case
    cases = [sweep_case(k) for k in range(ncases)]
    nodes = sum(c[0]["nx"] * c[0]["ny"] for c in cases)
    b = Batch(cases, device=0, storage=storage)
    b.tune(4)
    b.step(24)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(b.stream)
    b.step(steps)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    seq_steps = 24
    ev0.record(b.stream)
    b.step_sequential(seq_steps)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    ms_seq = ev0.elapsed_time(ev1) / seq_steps
    bad = sum(b.totals(i)["nonfinite"] for i in range(ncases))
    groups = b.groups()
    b.close()
    del b
    torch.cuda.empty_cache()
    if bad:
        print("bench: non-finite state in the sweep", file=sys.stderr)
        sys.exit(1)
    print(f"bench: sweep {ncases} grids {ms * 1e3:.1f} us/step batched, "
          f"{ms_seq * 1e3:.1f} us/step sequential", file=sys.stderr, flush=True)
    return {"value": round(ncases / (case_steps * ms * 1e-3), 3), "unit": "cases/s",
            "timed": f"{steps} consecutive steps of every case" +
                     (" (whole cases)" if steps >= case_steps else ""),
            "cases": ncases, "steps_per_case": case_steps, "nodes": nodes,
            "workload": "sweep_case(k), k < cases: side in {64,128,256,512}, sigma_T, "
                        "Stefan number, rho_s/rho_l, C0 drawn per case; 2D droplet",
            "storage": storage, "ms_per_step": round(ms, 6), "steps_timed": steps,
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1),
            "sequential": {"ms_per_step": round(ms_seq, 6), "steps_timed": seq_steps,
                           "value": round(ncases / (case_steps * ms_seq * 1e-3), 3)},
            "speedup_vs_sequential": round(ms_seq / ms, 3),
            "groups": groups}


def copy64_errors(forms) -> dict:
    """Per-field error of 5000 steps of the 64^3 copy of the 3D workload
    (drop radius 16, obstacle radius 3) in each storage form, against the
    FP64 oracle's fields at step 5000 stored in tests/golden (written by the
    script beside them), with the oracle's own spread under FP32-sized noise
    and the deviations of its two single-precision builds from the same file:
    max |gpu - oracle| / max |oracle| over fluid nodes."""
    from paper_2511_09422_amd.lbfz import Solver
    from paper_2511_09422_amd.workloads import droplet_3d
    ref = np.load(os.path.join(ROOT, "tests", "golden", "droplet3d_64_5000.npz"))
    names = [str(n) for n in ref["fields"]]
    cfg, phi, T, C, mask = droplet_3d(64, R=16.0, imp_R=3.0, seed=1)
    fluid = mask == 0
    out = {"workload": "64^3 copy of the 3D droplet, R=16, obstacle radius 3, 5000 steps",
           "oracle_spread": dict(zip(names, [float(f"{v:.3g}") for v in ref["spread"]])),
           "oracle_single_precision": dict(zip(names, [float(f"{v:.3g}")
                                                       for v in ref["dev_single"]])),
           "oracle_single_precision_weights_sum_to_one":
               dict(zip(names, [float(f"{v:.3g}") for v in ref["dev_single_cw"]]))}
    for f in forms:
        s = Solver(cfg, phi, T, C, mask=mask, device=0, storage=f)
        s.step(5000)
        got = s.fields()
        s.close()
        out[f] = {k: float(f"{np.abs(got[k][fluid] - ref[k][fluid]).max() / max(np.abs(ref[k][fluid]).max(), 1e-30):.3g}")
                  for k in names}
    return out


def unet_flops_per_image(S: int) -> float:
    """Multiply-adds x 2 of one forward pass of the surrogate U-Net on an
    S x S image (every convolution, padded channels included)."""
    from paper_2511_09422_amd import surrogate as sg
    return float(sum(2.0 * (S >> L.level) ** 2 * L.cout * L.taps * L.cin for L in sg.LAYERS))


def time_surrogate(iters: int, ngrids: int, warm: int, nacc: int) -> dict:
    """The learned surrogate screening a sweep: train on LB snapshot pairs of
    160 sweep seeds (25 snapshot levels of 256^2 grids, two input levels per
    pair), then on ngrids held-out seeds past `warm` strides of LB:
    one-stride predictions against the LB (accuracy per field, acceptance by
    the phase-field mass check, the check's false rejections of the LB's own
    pairs) over `nacc` strides, and the time of a screened stride (batched
    forward, LB on the rejected grids, restarts from the predicted fields)
    against the LB stride of all grids, medians over fresh copies of the
    held-out batch."""
    import torch
    from paper_2511_09422_amd import lbfz
    from paper_2511_09422_amd import surrogate as sg
    from paper_2511_09422_amd.workloads import sweep_case
    S = 256
    t0 = time.perf_counter()
    snaps, _ = sg.generate_snapshots(list(range(160)), S, 26)
    norm = sg.Normaliser(snaps)
    net = sg.UNet(sg.init_weights(0), 8, S)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sg.train(net, snaps, norm, iters, lr=1e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    npairs = snaps.shape[0] * (snaps.shape[1] - 1)
    del snaps
    torch.cuda.empty_cache()
    print(f"bench: surrogate trained, {iters} iterations in {t2 - t1:.1f} s "
          f"({(t2 - t1) / iters * 1e3:.2f} ms each)", file=sys.stderr, flush=True)
    cases = [sweep_case(k, side=S) for k in range(10000, 10000 + ngrids)]
    ref = lbfz.Batch(cases)
    ref.step((warm - 1) * sg.STRIDE)
    net_b = sg.UNet(net.weights(), ngrids, S)
    on_ref = sg.Screener(net_b, norm, ref)
    on_ref.observe()
    ref.step(sg.STRIDE)
    rows = []
    lb_res = []
    names = sg.FIELD_NAMES
    L = sg.nnlib()
    qsum = torch.zeros(ngrids, dtype=torch.float64, device=net_b.dev)
    after = torch.zeros((ngrids, sg.NEXP, S, S), dtype=torch.float32, device=net_b.dev)

    def rel(a, b):
        return float(np.linalg.norm(a.astype(np.float64) - b) /
                     max(np.linalg.norm(b.astype(np.float64)), 1e-30))
    for _ in range(nacc):
        res = on_ref.predict()
        pred = on_ref.pred.cpu().numpy()
        before_phi = on_ref.before[:, 0].double().sum(dim=(1, 2)).cpu().numpy()
        qb = on_ref.sums[on_ref.nsb + on_ref.nsa:on_ref.nsb + on_ref.nsa + ngrids].cpu().numpy()
        ref.step(sg.STRIDE)
        # the check on the LB's own pair (before, after the stride)
        ref.fields_all_to_device(sg.NEXP, after)
        sg._ck(L.lbfz_nn_phi_div_sums(sg._p(after), ngrids, sg.NEXP * S * S, S, S, 1, 0, 4, 5,
                                      sg._p(on_ref.parts), sg.PHI_DIV_PARTS, sg._p(qsum),
                                      net_b.st), "phi_div_sums")
        qa = qsum.cpu().numpy()
        after_phi = after[:, 0].double().sum(dim=(1, 2)).cpu().numpy()
        for i in range(ngrids):
            lb_res.append(sg.mass_residual(before_phi[i], after_phi[i], qb[i], qa[i], S * S))
        for i in range(ngrids):
            f = ref.fields(i, names)
            rows.append((res[i][0], [rel(pred[i, k], f[nm]) for k, nm in enumerate(names)
                                     if nm != "uz"]))
    acc = np.array([r[0] for r in rows])
    err = np.array([r[1] for r in rows])
    slow = err[:, :4].max(1)
    # timing, from the same LB states: the LB stride of all grids (graph
    # replays, HIP events), then a screened stride (host logic included: wall
    # clock around synchronised work), then a second screened stride, which
    # starts from partly restarted states (a rollout).  Medians over `reps`
    # fresh copies of the held-out batch (the code paths ran above).
    reps = 5
    lbs, scs, sc2s, accs, accs2 = [], [], [], [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for r in range(reps):
        scr = lbfz.Batch(cases)
        scr.step((warm - 1) * sg.STRIDE)
        on_scr = sg.Screener(net_b, norm, scr)
        on_scr.observe()   # the older input level: the LB stride timed next follows it
        torch.cuda.synchronize()
        ev0.record(scr.stream)
        scr.step(sg.STRIDE)
        ev1.record(scr.stream)
        torch.cuda.synchronize()
        lbs.append(ev0.elapsed_time(ev1))
        t3 = time.perf_counter()
        a1, _ = on_scr.stride()
        torch.cuda.synchronize()
        scs.append((time.perf_counter() - t3) * 1e3)
        t4 = time.perf_counter()
        a2, _ = on_scr.stride()
        torch.cuda.synchronize()
        sc2s.append((time.perf_counter() - t4) * 1e3)
        accs.append(np.mean(a1))
        accs2.append(np.mean(a2))
        bad = sum(scr.totals(i)["nonfinite"] for i in range(ngrids))
        scr.close()
        if bad:
            print("bench: non-finite LB state in the surrogate section", file=sys.stderr)
            sys.exit(1)
    lb_ms, sc_ms, sc2_ms = (float(np.median(v)) for v in (lbs, scs, sc2s))
    ev0.record(net_b.stream)
    net_b.forward()
    ev1.record(net_b.stream)
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1)
    flops = unet_flops_per_image(S) * ngrids
    bad = sum(ref.totals(i)["nonfinite"] for i in range(ngrids))
    ref.close()
    if bad:
        print("bench: non-finite LB state in the surrogate section", file=sys.stderr)
        sys.exit(1)
    print(f"bench: surrogate stride of {ngrids} grids: LB {lb_ms:.2f} ms, screened "
          f"{sc_ms:.2f} ms ({np.mean(accs):.2f} accepted; each copy "
          f"{' '.join(f'{v:.2f}' for v in scs)}), rollout {sc2_ms:.2f} ms, forward "
          f"{fwd_ms:.2f} ms", file=sys.stderr, flush=True)
    return {"value": round(lb_ms / sc_ms, 3), "unit": "x (LB-only stride time / screened)",
            "workload": f"{ngrids} held-out sweep seeds at {S}^2 after {warm} LB strides; "
                        f"stride {sg.STRIDE} steps; U-Net 32/64/128, BF16 MFMA",
            "train": {"pairs": npairs, "iterations": iters, "batch": 8,
                      "ms_per_iteration": round((t2 - t1) / iters * 1e3, 2),
                      "data_s": round(t1 - t0, 1)},
            "timing": f"medians over {reps} copies of the held-out batch",
            "lb_stride_ms": round(lb_ms, 3), "screened_stride_ms": round(sc_ms, 3),
            "screened_accepted": round(float(np.mean(accs)), 3),
            "rollout_stride": {"ms": round(sc2_ms, 3), "accepted": round(float(np.mean(accs2)), 3),
                               "speedup": round(lb_ms / sc2_ms, 3)},
            "one_stride": {"predictions": len(rows), "accepted": round(float(acc.mean()), 3),
                           "mass_tol": sg.MASS_TOL,
                           "lb_pairs_rejected": round(float((np.array(lb_res) > sg.MASS_TOL).mean()), 3),
                           "lb_pair_residual_median": float(f"{np.median(lb_res):.3g}"),
                           "accepted_all_slow_within_1e-2": round(float((slow[acc] <= 1e-2).mean()), 3),
                           "accepted_slow_max_p90": round(float(np.percentile(slow[acc], 90)), 5),
                           "median_rel_l2": dict(zip([n for n in names if n != "uz"],
                                                     np.median(err, 0).round(5).tolist()))},
            "forward": {"ms": round(fwd_ms, 3), "images": ngrids,
                        "roofline": {"bound": "mfma", "achieved": round(flops / fwd_ms / 1e9, 1),
                                     "peak": 2500.0, "unit": "TFLOP/s",
                                     "frac": round(flops / fwd_ms / 1e9 / 2500.0, 4),
                                     "gflop_per_image": round(unet_flops_per_image(S) / 1e9, 3)}}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=sorted(POP_BYTES),
                    help="population storage of the headline figure")
    ap.add_argument("--forms", default="f16,bf16",
                    help="other storage forms timed on the same workload ('' for none)")
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--n3d", type=int, default=256,
                    help="side of the 3D droplet workload timed alongside (0: skip)")
    ap.add_argument("--steps3d", type=int, default=200)
    ap.add_argument("--no-error-64", action="store_true",
                    help="skip the 5000-step per-field error of the 64^3 copy (profiling runs, "
                         "which should see only the 256^3 launches of the 3D kernels)")
    ap.add_argument("--sweep-cases", type=int, default=512,
                    help="grids of the batched parameter sweep timed alongside (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=10000,
                    help="batched steps timed (default: one whole case)")
    ap.add_argument("--sweep-case-steps", type=int, default=10000,
                    help="steps that make one sweep case (cases/s is quoted for this length)")
    ap.add_argument("--surrogate-iters", type=int, default=12000,
                    help="training iterations of the surrogate (0: skip the surrogate section)")
    ap.add_argument("--surrogate-grids", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_09422_amd.workloads import droplet_2d

    n = args.n
    cfg, phi, T, C = droplet_2d(n, n, R=n / 4.0, seed=0)
    forms = [f for f in args.forms.split(",") if f and f != args.storage]
    for f in forms:
        if f not in POP_BYTES:
            print(f"bench.py: unknown storage form {f}", file=sys.stderr)
            sys.exit(2)
    print(f"bench: 2D droplet {n}x{n}, storage {args.storage} (+ {forms}), warmup "
          f"{args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    main_r = time_form(cfg, phi, T, C, args.storage, args.warmup, args.steps)
    print(f"bench: {args.storage} {main_r['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr,
          flush=True)
    copy_r = time_copy(main_r["bytes_per_node"] * n * n)
    print(f"bench: copy of the same {copy_r['bytes'] / 1e6:.0f} MB {copy_r['us']:.2f} us "
          f"({copy_r['GBs']:.0f} GB/s)", file=sys.stderr, flush=True)
    pat_r = time_pattern(n)
    print(f"bench: the step's plane pattern {pat_r['us']:.2f} us ({pat_r['GBs']:.0f} GB/s)",
          file=sys.stderr, flush=True)
    other = {}
    for f in forms:
        r = time_form(cfg, phi, T, C, f, args.warmup, args.steps)
        print(f"bench: {f} {r['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr, flush=True)
        other[f] = {"value": round(r["mlups"], 2), "unit": "MLUPS",
                    "ms_per_step": round(r["ms_per_step"], 6),
                    "speedup_vs_" + args.storage: round(main_r["ms_per_step"] / r["ms_per_step"], 3),
                    "roofline": {"bound": "hbm", "achieved": round(r["achieved"], 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(r["achieved"] / HBM_PEAK_GBS, 4),
                                 "bytes_per_node": r["bytes_per_node"],
                                 "design_bytes_per_node": r["design_bytes_per_node"],
                                 "frac_at_design_bytes":
                                     round(r["design_GBs"] / HBM_PEAK_GBS, 4),
                                 "traffic": load_traffic(f"k_step2d_{f}_{n}")}}
    droplet3d = None
    if args.n3d:
        from paper_2511_09422_amd.workloads import droplet_3d
        m = args.n3d
        cfg3, phi3, T3, C3, mask3 = droplet_3d(m, R=m / 4.0, imp_R=12.0 * m / 256.0, seed=1)
        forms3 = {}
        base3 = None
        for f in [args.storage] + forms:
            r = time_form(cfg3, phi3, T3, C3, f, max(1, args.warmup // 10), args.steps3d,
                          mask=mask3)
            print(f"bench: 3D {f} {r['ms_per_step'] * 1e3:.1f} us/step", file=sys.stderr,
                  flush=True)
            if base3 is None:
                base3 = r
            forms3[f] = {"value": round(r["mlups"], 2), "unit": "MLUPS",
                         "ms_per_step": round(r["ms_per_step"], 6),
                         "speedup_vs_" + args.storage:
                             round(base3["ms_per_step"] / r["ms_per_step"], 3),
                         "roofline": {"bound": "hbm", "achieved": round(r["achieved"], 1),
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": round(r["achieved"] / HBM_PEAK_GBS, 4),
                                      "bytes_per_node": r["bytes_per_node"],
                                      "traffic": load_traffic(f"k_step3d_{f}_{m}")}}
        droplet3d = {"workload": f"3D droplet freezing {m}^3, R={m // 4}, obstacle radius "
                                 f"{12 * m // 256}, D3Q19+3xD3Q7, FP32 arithmetic",
                     "steps": args.steps3d, "forms": forms3}
        pat3 = time_pattern3d(m)
        if "f32" in forms3:
            pat3["step_vs_pattern"] = round(pat3["us"] * 1e-3 / forms3["f32"]["ms_per_step"], 4)
        droplet3d["step_pattern"] = dict(kernel="lbfz_stream_planes3d", **pat3)
        print(f"bench: 3D plane pattern {pat3['us']:.1f} us ({pat3['GB/s']:.0f} GB/s, "
              f"{pat3['bytes_per_node']} B/node)", file=sys.stderr, flush=True)
        if not args.no_error_64:
            droplet3d["error_vs_oracle_64"] = copy64_errors([args.storage] + forms)
            print("bench: 3D 64^3 copy, 5000 steps, error vs oracle: " +
                  json.dumps(droplet3d["error_vs_oracle_64"]), file=sys.stderr, flush=True)
    sweep = None
    if args.sweep_cases:
        sweep = time_sweep(args.sweep_cases, args.sweep_steps, args.sweep_case_steps,
                           args.storage)
    surrogate = None
    if args.surrogate_iters:
        surrogate = time_surrogate(args.surrogate_iters, args.surrogate_grids, 8, 3)
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    out = {
        "metric": "coupled-field MLUPS (FP32 vs FP16-store); sweep cases/s; surrogate speedup",
        "value": round(main_r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D droplet freezing {n}x{n}, R={n // 4}, interface width 4, "
                               "D2Q9+3xD2Q5, FP32 arithmetic",
                   "grid": [n, n], "storage": args.storage,
                   "bytes_per_node": main_r["bytes_per_node"],
                   "wall_s": round(main_r["wall"], 3)},
        "roofline": {"bound": "hbm", "achieved": round(main_r["achieved"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(main_r["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(f"k_step2d_{args.storage}_{n}")},
        "copy_ceiling": {"kernel": "lbfz_stream_copy", "bytes": copy_r["bytes"],
                         "us": round(copy_r["us"], 2), "GB/s": round(copy_r["GBs"], 1),
                         "frac_of_peak": round(copy_r["GBs"] / HBM_PEAK_GBS, 4),
                         "step_vs_copy": round(main_r["achieved"] / copy_r["GBs"], 4),
                         "runtime_copy": {"us": round(copy_r["runtime_copy_us"], 2),
                                          "GB/s": round(copy_r["runtime_copy_GBs"], 1)},
                         "step_pattern": {"kernel": "lbfz_stream_planes", "bytes": pat_r["bytes"],
                                          "us": round(pat_r["us"], 2),
                                          "GB/s": round(pat_r["GBs"], 1),
                                          "frac_of_peak": round(pat_r["GBs"] / HBM_PEAK_GBS, 4),
                                          "step_vs_pattern":
                                              round(main_r["achieved"] / pat_r["GBs"], 4)}},
    }
    if other:
        out["storage_forms"] = other
    if droplet3d:
        out["droplet3d"] = droplet3d
    if sweep:
        out["sweep"] = sweep
    if surrogate:
        out["surrogate"] = surrogate
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, phi, T, C)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
