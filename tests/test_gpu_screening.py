"""The learned surrogate against the plain LB on held-out sweep seeds (its
use: screening a sweep 64 steps at a time, with the LB as fallback and judge).

A network trained on the GPU by the project's own kernels (8000 iterations
of batch 8 on the 4000 LB snapshot pairs of 160 sweep seeds, under a minute)
predicts 64 steps ahead from LB states of
16 other seeds, past the initial transient (strides 8-11).  Checked:
  - it beats the no-change baseline on every slow field (phi, f_l, T, C);
  - the phase-field mass check (residual <= 1e-3) accepts a fair share, and
    at least 90% of the accepted predictions are within relative L2 1e-2 of
    the LB on every slow field (the error bar of the screened sweep).
The time of a screened stride (one batched forward, the LB on the rejected
grids, restarts of the accepted ones) against the LB stride of all grids is
reported (bench.py measures it on 64 grids).
The velocity is reported, not gated: 64 steps ahead it is dominated by the
flow's acoustic and interface currents, which one snapshot does not determine
(the no-change prediction is further from it than zero is); accepted grids
restart at rest.  The check's false-reject rate on the LB's own states (the
residual of each LB pair before / after a stride) is reported beside it."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SLOW = ("phi", "fl", "T", "C")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_screening_against_the_lb_on_held_out_seeds():
    import torch
    from paper_2511_09422_amd import lbfz
    from paper_2511_09422_amd import surrogate as sg
    from paper_2511_09422_amd.workloads import sweep_case
    S, NG, WARM, NSTR = 256, 16, 8, 4
    t0 = time.time()
    snaps, _ = sg.generate_snapshots(list(range(160)), S, 26)
    norm = sg.Normaliser(snaps)
    net = sg.UNet(sg.init_weights(0), 8, S)
    sg.train(net, snaps, norm, 8000, lr=1e-3)
    torch.cuda.synchronize()
    print(f"[screen] trained in {time.time() - t0:.1f} s", flush=True)
    del snaps
    cases = [sweep_case(k, side=S) for k in range(10000, 10000 + NG)]
    ref = lbfz.Batch(cases)
    ref.step(WARM * sg.STRIDE)
    netB = sg.UNet(net.weights(), NG, S)
    scr = sg.Screener(netB, norm, ref)
    rows = []
    for _ in range(NSTR):
        res = scr.predict()
        before = scr.before[:, :sg.NF].cpu().numpy()
        pred = scr.pred.cpu().numpy()
        ref.step(sg.STRIDE)
        for i in range(NG):
            f = ref.fields(i, ("phi", "fl", "T", "C", "ux", "uy"))
            truth = [f[k] for k in ("phi", "fl", "T", "C", "ux", "uy")]
            # the check applied to the LB's own pair (before, after the stride)
            lb_r = sg.mass_residual(before[i, 0].sum(dtype=np.float64), truth[0].sum(dtype=np.float64),
                                    before[i, 1].sum(dtype=np.float64), truth[1].sum(dtype=np.float64),
                                    S * S, scr.ratios[i])
            rows.append((res[i][0], [_rel(pred[i, k], truth[k]) for k in range(6)],
                         [_rel(before[i, k], truth[k]) for k in range(6)], lb_r))
    acc = np.array([r[0] for r in rows])
    err = np.array([r[1] for r in rows])
    base = np.array([r[2] for r in rows])
    med, bmed = np.median(err, 0), np.median(base, 0)
    slow = err[:, :4].max(1)
    lb_res = np.array([r[3] for r in rows])
    print(f"[screen] the check on the LB's own pairs: residual median {np.median(lb_res):.2e}, "
          f"p95 {np.percentile(lb_res, 95):.2e}; rejected at {sg.MASS_TOL:g}: "
          f"{(lb_res > sg.MASS_TOL).mean():.2f}", flush=True)
    print(f"[screen] median rel L2 surrogate {dict(zip(sg.FIELD_NAMES, med.round(5)))}", flush=True)
    print(f"[screen] median rel L2 no-change {dict(zip(sg.FIELD_NAMES, bmed.round(5)))}", flush=True)
    print(f"[screen] accepted {acc.mean():.2f}; accepted within 1e-2: "
          f"{(slow[acc] <= 1e-2).mean():.3f}; p90 {np.percentile(slow[acc], 90):.4f}", flush=True)
    for k in range(4):
        assert med[k] < bmed[k], (SLOW[k], med[k], bmed[k])
    assert acc.mean() >= 0.25
    assert (slow[acc] <= 1e-2).mean() >= 0.9
    # one screened stride against the LB stride of every grid (same grids,
    # continued from the current level)
    other = lbfz.Batch(cases)
    other.step((WARM + NSTR) * sg.STRIDE)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    other.step(sg.STRIDE)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    accs, _ = scr.stride()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    lb_ms, sc_ms = (t2 - t1) * 1e3, (t3 - t2) * 1e3
    print(f"[screen] stride of {NG} grids: LB {lb_ms:.2f} ms, screened {sc_ms:.2f} ms "
          f"({np.mean(accs):.2f} accepted), gain {lb_ms / sc_ms:.2f}x", flush=True)
    for i in range(NG):
        assert ref.totals(i)["nonfinite"] == 0
    ref.close()
    other.close()
