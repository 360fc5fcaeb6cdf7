"""16-bit population storage (FP16 / BF16 offsets, FP32 arithmetic) against
the FP64 oracle, through the C ABI.

A moving population is stored as round16((v - w_i r) S) with r the reference
moment of the node it is stored at (phi, 3 p, (rho c)_ref T, C of the writing
step; p one level earlier) and S a power of two, and read back as
w_i r + s / S.  One step therefore adds at most u |v - w_i r| per moving
population to the FP32 rounding, u the unit roundoff of the format (2^-11
FP16, 2^-8 BF16); the one-step test checks that bound element by element.
The rest populations are FP32.  Over many steps the quantisation acts like
noise of that size; the long-run errors against the FP64 oracle are printed
and bounded loosely (the bound is a regression guard, the printed values are
the measurement).
"""
import numpy as np
import pytest

from oracle.lbref import Oracle
from paper_2511_09422_amd.lbfz import Solver
from tests.test_gpu_parity import CASES, FIELDS, THREADS, _load_into_oracle, rel_linf

pytestmark = pytest.mark.gpu

UNIT = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
W5 = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
SETS = (("f", slice(0, 5), 0, W5), ("g", slice(5, 14), 1, W9), ("h", slice(14, 19), 2, W5),
        ("l", slice(19, 24), 3, W5))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", ["64x64", "walls"])
def test_initial_state_equals_fp32(storage, case):
    """Every moving population starts at its reference (offset 0), so the
    decoded initial state is the FP32 one bit for bit."""
    cfg, phi, T, C = CASES[case]()
    a = Solver(cfg, phi, T, C, storage="f32").get_state()
    b = Solver(cfg, phi, T, C, storage=storage).get_state()
    assert np.array_equal(a[:24], b[:24])
    assert np.array_equal(a[24:28], b[24:28])


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case,K", [("64x64", 0), ("64x64", 300), ("150x37", 100),
                                    ("periodic", 100), ("walls", 200)])
def test_one_step_quantisation_bound(storage, case, K):
    _one_step_check(storage, case, K, *CASES[case]())


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_one_step_quantisation_bound_full_size(storage):
    """The same bound on the 2048^2 droplet (radius 512) in the benchmark's
    launch configuration, after 200 steps."""
    from paper_2511_09422_amd.workloads import droplet_2d
    _one_step_check(storage, "2048x2048", 200, *droplet_2d(2048, 2048, R=512.0, seed=0))


def _one_step_check(storage, case, K, cfg, phi, T, C):
    print(f"[16bit one-step] {storage} {case} after {K} steps", flush=True)
    s = Solver(cfg, phi, T, C, storage=storage)
    s.step(K)
    st0 = s.get_state().astype(np.float64)
    o = _load_into_oracle(cfg, st0, s.shape)
    lev = o.fields()            # moments of the level the step starts from
    refs = {"f": lev["phi"], "g": 3.0 * st0[25], "h": cfg["rhoc_ref"] * lev["T"],
            "l": lev["C"]}
    s.step(1)
    o.step(1)
    got = s.get_state().astype(np.float64)
    u = UNIT[storage]
    worst = {}
    for name, sl, w, wts in SETS:
        ref = o.get_pops(w)
        tol32 = 2e-5 * np.abs(ref).max()
        err = np.abs(got[sl] - ref)
        assert err[0].max() <= tol32, (storage, case, K, name, "rest", err[0].max())
        off = np.abs(ref[1:] - wts[1:, None, None] * refs[name][None])
        bound = u * off + tol32
        ratio = (err[1:] / bound).max()
        worst[name] = ratio
        assert ratio <= 1.0, (storage, case, K, name, ratio)
    for k, w in ((24, 0), (25, 1), (26, 2), (27, 3), (28, 5), (29, 6)):
        assert rel_linf(got[k], o.get_state(w)) <= 2e-5, (storage, case, K, "state", k)
    f, r = s.fields(), o.fields()
    errs = {k: rel_linf(f[k], r[k]) for k in FIELDS}
    print(f"[16bit one-step] {storage} {case} K={K} err/bound " +
          " ".join(f"{k}={v:.2f}" for k, v in worst.items()) + " | fields " +
          " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)


LONG_BOUND = {"f16": 2e-2, "bf16": 1.5e-1}


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_droplet_64x64_1000_steps_error(storage):
    """Per-field error of the 1000-step 64x64 droplet against the FP64 oracle,
    and the phase-field budget sum_f - sum_f(0) - M_pc."""
    cfg, phi, T, C = CASES["64x64"]()
    s = Solver(cfg, phi, T, C, storage=storage)
    t0 = s.totals()
    s.step(1000)
    got = s.fields()
    t1 = s.totals()
    o = Oracle(cfg, phi, T, C, threads=THREADS)
    o.step(1000)
    ref = o.fields()
    errs = {k: rel_linf(got[k], ref[k]) for k in FIELDS}
    budget = (t1["sum_f"] - t0["sum_f"] - t1["mpc"]) / (phi.size)
    print(f"[16bit long] {storage} 1000 steps " + " ".join(f"{k}={v:.2e}" for k, v in errs.items())
          + f" | phase-field budget per node {budget:.2e} nonfinite {t1['nonfinite']}", flush=True)
    assert t1["nonfinite"] == 0
    if storage != "f32":
        for k, e in errs.items():
            assert e <= LONG_BOUND[storage], (storage, k, e)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_state_round_trip(storage):
    """get_state -> set_state re-encodes against the imported phi, C (same
    references: f and l come back to FP32 rounding) and against p and the
    mapped T (g and h come back within the quantisation bound)."""
    cfg, phi, T, C = CASES["150x37"]()
    s = Solver(cfg, phi, T, C, storage=storage)
    s.step(150)
    a = s.get_state().astype(np.float64)
    s.set_state(a.astype(np.float32))
    b = s.get_state().astype(np.float64)
    u = UNIT[storage]
    for name, sl, _, _ in SETS:
        scale = np.abs(a[sl]).max()
        tol = 1e-6 * scale if name in ("f", "l") else u * scale
        assert np.abs(b[sl] - a[sl]).max() <= tol, (storage, name)
    assert np.array_equal(a[24:], b[24:])
    s.step(10)
    assert s.totals()["nonfinite"] == 0
