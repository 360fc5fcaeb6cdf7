"""Writes droplet3d_64_5000.npz beside this script: the FP64 oracle's
macroscopic fields after 5000 steps of the 64^3 copy of the 3D droplet
workload (drop radius 16 on the cold wall, obstacle radius 3 at the seeded
offset scaled by 1/4, interface width 4), stored as float32, plus the
spread of the same oracle run whose populations carry FP32-sized relative
noise (uniform, 6e-8) before every step: max |noisy - clean| / max |clean|
per field, and the deviation of the oracle's own single-precision build
(variant "single": the same source with every double a float) from it
after the same 5000 steps -- what evaluating the scheme in FP32 does to
this trajectory -- and that of the single-precision build whose weights sum
to one in FP32 (variant "single_cw").  It calls only the oracle and the
seeded input generator.

    python tests/golden/make_droplet3d_64_5000.py [threads] [--single-only]

--single-only adds the two single-precision deviations to an existing file.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.lbref import Oracle  # noqa: E402
from paper_2511_09422_amd.workloads import droplet_3d  # noqa: E402

FIELDS = ("phi", "fl", "T", "C", "ux", "uy", "uz", "p")
STEPS = 5000
NOISE = 6e-8


def single_deviation(cfg, phi, T, C, mask, ref, threads: int,
                     variant: str = "single") -> np.ndarray:
    """max |single - FP64| / max |FP64| over fluid nodes, per field, after
    STEPS steps of one of the oracle's single-precision builds."""
    fluid = mask == 0
    o = Oracle(cfg, phi, T, C, mask=mask, threads=threads, variant=variant)
    o.step(STEPS)
    f = o.fields()
    return np.array([float(np.abs(f[k][fluid] - ref[k][fluid]).max() /
                           max(np.abs(ref[k][fluid]).max(), 1e-30)) for k in FIELDS])


def main(threads: int, single_only: bool = False) -> None:
    cfg, phi, T, C, mask = droplet_3d(64, R=16.0, imp_R=3.0, seed=1)
    fluid = mask == 0
    path = os.path.join(HERE, "droplet3d_64_5000.npz")
    if single_only:
        old = dict(np.load(path))
        ref = {f: old[f].astype(np.float64) for f in FIELDS}
        old["dev_single"] = single_deviation(cfg, phi, T, C, mask, ref, threads)
        old["dev_single_cw"] = single_deviation(cfg, phi, T, C, mask, ref, threads, "single_cw")
        np.savez_compressed(path, **old)
        for k in ("dev_single", "dev_single_cw"):
            print(k + " " + " ".join(f"{f}={v:.2e}" for f, v in zip(FIELDS, old[k])))
        return
    t0 = time.time()
    o = Oracle(cfg, phi, T, C, mask=mask, threads=threads)
    for k in range(0, STEPS, 500):
        o.step(500)
        print(f"clean {k + 500} steps, {time.time() - t0:.0f} s", flush=True)
    ref = o.fields()
    tot = o.totals()
    del o
    rng = np.random.default_rng(7)
    o = Oracle(cfg, phi, T, C, mask=mask, threads=threads)
    for k in range(STEPS):
        for w in range(4):
            p = o.get_pops(w)
            o.set_pops(w, p * (1.0 + NOISE * rng.uniform(-1.0, 1.0, size=p.shape)))
        o.step(1)
        if (k + 1) % 500 == 0:
            print(f"noisy {k + 1} steps, {time.time() - t0:.0f} s", flush=True)
    noisy = o.fields()
    spread = {}
    for f in FIELDS:
        scale = max(np.abs(ref[f][fluid]).max(), 1e-30)
        spread[f] = float(np.abs(noisy[f][fluid] - ref[f][fluid]).max() / scale)
    out = {f: ref[f].astype(np.float32) for f in FIELDS}
    out["spread"] = np.array([spread[f] for f in FIELDS])
    out["fields"] = np.array(FIELDS)
    out["totals"] = np.array([tot["sum_f"], tot["sum_l"], tot["sum_h"], tot["mpc"],
                              tot["vol_solid"], tot["vol_sl"]])
    out["dev_single"] = single_deviation(cfg, phi, T, C, mask, ref, threads)
    out["dev_single_cw"] = single_deviation(cfg, phi, T, C, mask, ref, threads, "single_cw")
    np.savez_compressed(path, **out)
    print("spread " + " ".join(f"{f}={spread[f]:.2e}" for f in FIELDS), flush=True)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    main(int(args[0]) if args else 8, "--single-only" in sys.argv)
