"""3D step with 16-bit population storage (FP16 / BF16 offsets from the
reference moments, FP32 arithmetic) against the FP64 oracle, through the C
ABI; the same bars as the 2D 16-bit tests (one step: every moving population
within u |v - w_i r| of the oracle, u the format's unit roundoff; long runs:
printed per-field errors under a loose regression bound)."""
import os

import numpy as np
import pytest

from oracle.lbref import Oracle
from paper_2511_09422_amd.lbfz import Solver
from paper_2511_09422_amd.workloads import droplet_3d
from tests.test_gpu_parity3d import CASES, FIELDS, THREADS, _oracle_from_state, rel_linf

pytestmark = pytest.mark.gpu

UNIT = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
W7 = np.array([0.0] + [1 / 6] * 6)
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
SETS = (("f", slice(0, 7), 0, W7), ("g", slice(7, 26), 1, W19), ("h", slice(26, 33), 2, W7),
        ("l", slice(33, 40), 3, W7))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", ["drop16", "box40x20x70", "ragged70x13x11"])
def test_initial_state_equals_fp32_3d(storage, case):
    cfg, phi, T, C, mask = CASES[case]()
    a = Solver(cfg, phi, T, C, mask=mask, storage="f32").get_state()
    b = Solver(cfg, phi, T, C, mask=mask, storage=storage).get_state()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case,K", [("drop16", 0), ("drop16", 60), ("box40x20x70", 40),
                                    ("periodic", 40), ("ragged70x13x11", 30)])
def test_one_step_quantisation_bound_3d(storage, case, K):
    cfg, phi, T, C, mask = CASES[case]()
    print(f"[3d 16bit one-step] {storage} {case} K={K}", flush=True)
    s = Solver(cfg, phi, T, C, mask=mask, storage=storage)
    s.step(K)
    st0 = s.get_state().astype(np.float64)
    o = _oracle_from_state(cfg, st0, s.shape, mask)
    lev = o.fields()
    refs = {"f": lev["phi"], "g": 3.0 * st0[41], "h": cfg["rhoc_ref"] * lev["T"], "l": lev["C"]}
    s.step(1)
    o.step(1)
    got = s.get_state().astype(np.float64)
    fluid = (mask == 0) if mask is not None else np.ones(s.shape, bool)
    u = UNIT[storage]
    worst = {}
    for name, sl, w, wts in SETS:
        ref = o.get_pops(w)
        err = np.abs(got[sl] - ref)
        off = np.abs(ref - wts[:, None, None, None] * refs[name][None])
        keep = np.ones(s.shape, bool) if name == "h" else fluid
        tol32 = 2e-5 * np.abs(ref[:, keep]).max()
        # rest components: FP32 (g0, h0) or identically zero (f0, l0)
        assert err[0][keep].max() <= tol32, (storage, case, K, name, "rest")
        ratio = (err[1:][:, keep] / (u * off[1:][:, keep] + tol32)).max()
        worst[name] = ratio
        assert ratio <= 1.0, (storage, case, K, name, ratio)
    f, r = s.fields(), o.fields()
    errs = {k: rel_linf(f[k], r[k], mask) for k in FIELDS}
    print(f"[3d 16bit one-step] {storage} {case} K={K} err/bound " +
          " ".join(f"{k}={v:.2f}" for k, v in worst.items()) + " | fields " +
          " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)


LONG_BOUND = {"f16": 2e-2, "bf16": 1.5e-1}


def _state3d(o, shape):
    """Oracle populations and previous-level fields in the GPU state layout."""
    st = np.zeros((47,) + tuple(shape))
    for w, sl in ((0, slice(0, 7)), (1, slice(7, 26)), (2, slice(26, 33)), (3, slice(33, 40))):
        st[sl] = o.get_pops(w)
    for k in range(7):
        st[40 + k] = o.get_state(k)
    return st


def _dev_spread(cfg, st0, shape, mask, steps, ref, dev, seeds=(1, 2, 3)):
    """Spread of the FP64 oracle started from st0 when every population and
    previous-level value is moved by dev * U(-1, 1) before each step."""
    spread = {k: 0.0 for k in FIELDS}
    for sd in seeds:
        rng = np.random.default_rng(sd)
        o = _oracle_from_state(cfg, st0, shape, mask)
        for _ in range(steps):
            st = _state3d(o, shape) + dev * rng.uniform(-1, 1, size=dev.shape)
            for w, sl in ((0, slice(0, 7)), (1, slice(7, 26)), (2, slice(26, 33)),
                          (3, slice(33, 40))):
                o.set_pops(w, st[sl])
            for k in range(7):
                o.set_state(k, st[40 + k])
            o.step(1)
        f = o.fields()
        for k in FIELDS:
            spread[k] = max(spread[k], rel_linf(f[k], ref[k], mask))
    return spread


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_3d_64_copy_100_steps_error(storage):
    """Per-field error of 100 steps of the 64^3 copy of the 3D workload
    against the FP64 oracle, and the phase-field budget."""
    cfg, phi, T, C, mask = droplet_3d(64, R=16.0, imp_R=3.0, seed=1)
    s = Solver(cfg, phi, T, C, mask=mask, storage=storage)
    t0 = s.totals()
    if storage == "f32":
        # the GPU's one-step deviation from the oracle at every entry, held to
        # the one-step bar, then used as the per-step perturbation of the
        # oracle whose spread sets the 100-step bar
        st0 = s.get_state().astype(np.float64)
        o1 = _oracle_from_state(cfg, st0, s.shape, mask)
        s.step(1)
        o1.step(1)
        dev = np.abs(s.get_state().astype(np.float64) - _state3d(o1, s.shape))
        ost = _state3d(o1, s.shape)
        for name, sl in (("f", slice(0, 7)), ("g", slice(7, 26)), ("h", slice(26, 33)),
                         ("l", slice(33, 40))) + tuple((f"state{k}", slice(k, k + 1))
                                                       for k in range(40, 47)):
            worst = dev[sl].max() / max(np.abs(ost[sl]).max(), 1e-30)
            assert worst <= 2e-5, (name, worst)
        del o1
        s.step(99)
    else:
        s.step(100)
    got = s.fields()
    t1 = s.totals()
    o = Oracle(cfg, phi, T, C, mask=mask, threads=THREADS)
    o.step(100)
    ref = o.fields()
    errs = {k: rel_linf(got[k], ref[k], mask) for k in FIELDS}
    budget = (t1["sum_f"] - t0["sum_f"] - t1["mpc"]) / phi.size
    print(f"[3d 16bit long] {storage} 100 steps " +
          " ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f" | phase-field budget per node {budget:.2e}", flush=True)
    assert t1["nonfinite"] == 0
    if storage == "f32":
        # FP32 storage is held to 1e-4, or three times the spread of the FP64
        # oracle perturbed before every step by the GPU's own (bounded)
        # one-step deviation, or 1.25 times the deviation of the oracle's own
        # single-precision build after the same 100 steps (what evaluating the
        # scheme in FP32 does by itself; two FP32 evaluations with different
        # rounding sequences land within 10 % of each other)
        spread = _dev_spread(cfg, st0, s.shape, mask, 100, ref, dev)
        o32 = Oracle(cfg, phi, T, C, mask=mask, threads=THREADS, variant="single")
        o32.step(100)
        r32 = o32.fields()
        dev32 = {k: rel_linf(r32[k], ref[k], mask) for k in FIELDS}
        print("[3d 16bit long] f32 oracle spread " +
              " ".join(f"{k}={v:.2e}" for k, v in spread.items()) + " | single-precision oracle " +
              " ".join(f"{k}={v:.2e}" for k, v in dev32.items()), flush=True)
        for k, e in errs.items():
            assert e <= max(1e-4, 3.0 * spread[k], 1.25 * dev32[k]), (storage, k, e, spread[k],
                                                                        dev32[k])
    else:
        # 16-bit storage: a regression guard on the stated per-field errors
        for k, e in errs.items():
            assert e <= LONG_BOUND[storage], (storage, k, e)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_state_round_trip_3d(storage):
    cfg, phi, T, C, mask = CASES["drop16"]()
    s = Solver(cfg, phi, T, C, mask=mask, storage=storage)
    s.step(40)
    a = s.get_state().astype(np.float64)
    s.set_state(a.astype(np.float32))
    b = s.get_state().astype(np.float64)
    u = UNIT[storage]
    for name, sl, _, _ in SETS:
        scale = np.abs(a[sl]).max()
        tol = 1e-6 * scale if name in ("f", "l") else u * scale
        assert np.abs(b[sl] - a[sl]).max() <= tol, (storage, name)
    assert np.array_equal(a[40:], b[40:])
    s.step(5)
    assert s.totals()["nonfinite"] == 0


GOLDEN_5000 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "droplet3d_64_5000.npz")


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_3d_64_copy_5000_steps_against_stored_oracle(storage):
    """The 64^3 copy of the 3D workload (drop radius 16, obstacle radius 3)
    after 5000 steps against the FP64 oracle's fields at step 5000, stored by
    tests/golden/make_droplet3d_64_5000.py (which calls only the oracle),
    with three references stored beside them: the spread of the same oracle
    under FP32-sized noise, and the deviations after the same 5000 steps of
    two single-precision builds of the oracle, one with every double a float
    (phi 9e-3, u_x 0.18) and one whose lattice weights also sum to one in
    FP32 (rest weights the complements of the moving ones; the D3Q7 +-z pair
    one ulp below fl(1/6), as the GPU kernels take them: phi 5.5e-3, u_x
    1.2e-2).  After 5000 steps the trajectory's sensitivity to FP32
    evaluation dominates, and the second build is the FP32 evaluation of
    this scheme.  FP32 storage: within max(1e-4, 3 x the spread, 1.5 x that
    build's deviation) per field (measured GPU / build ratios 0.93-1.00).
    FP16 storage: within 2.5 x that build's deviation (measured at most
    1.64, u_y).  BF16 storage (8-bit significand) is held to a guard against
    blow-ups (measured u 0.2, phi 2.2e-2)."""
    ref = np.load(GOLDEN_5000)
    names = [str(n) for n in ref["fields"]]
    spread = dict(zip(names, ref["spread"].tolist()))
    dev32 = dict(zip(names, ref["dev_single"].tolist()))
    dev_cw = dict(zip(names, ref["dev_single_cw"].tolist()))
    cfg, phi, T, C, mask = droplet_3d(64, R=16.0, imp_R=3.0, seed=1)
    print(f"[3d 5000] {storage}", flush=True)
    s = Solver(cfg, phi, T, C, mask=mask, storage=storage)
    s.step(5000)
    got = s.fields()
    errs = {k: rel_linf(got[k], ref[k].astype(np.float64), mask) for k in names}
    print(f"[3d 5000] {storage} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          " | oracle spread " + " ".join(f"{k}={v:.2e}" for k, v in spread.items()) +
          " | single-precision oracle " + " ".join(f"{k}={v:.2e}" for k, v in dev32.items()) +
          " | the same, weights summing to one " +
          " ".join(f"{k}={v:.2e}" for k, v in dev_cw.items()), flush=True)
    assert s.totals()["nonfinite"] == 0
    for k, e in errs.items():
        if storage == "f32":
            assert e <= max(1e-4, 3.0 * spread[k], 1.5 * dev_cw[k]), (k, e, spread[k], dev_cw[k])
        elif storage == "f16":
            assert e <= 2.5 * dev_cw[k], (storage, k, e, dev_cw[k])
        else:
            assert e <= 0.5, (storage, k, e)
