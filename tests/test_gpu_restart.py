"""Equilibrium restart from macroscopic fields and subset stepping of a
batch (the two halves of the surrogate screening's LB fallback).

Restart: populations at the equilibria of (phi, f_l, T, C, u, p) drop the
non-equilibrium parts and the interface force's half-step, so a restart from a
solver's own fields reproduces those fields to the size of those parts (a
first GPU run measured phi, f_l, C within 1e-4 and T within 1e-3 relative L2;
the bars are 3x that), and 64 steps run on from a restart stay close to 64
steps of the original: the slow fields within 1e-2 (the screening's accuracy
bar).  The velocity and the pressure carry the dropped parts and are only
checked to stay finite and bounded.

Subset stepping: a grid's step in the batch kernel does not depend on which
other grids share the launch, so the selected grids match a batch that steps
every grid bit for bit; the grids left out are stale (reads and steps refused)
until restarted."""
import numpy as np
import pytest

from paper_2511_09422_amd.workloads import droplet_2d, sweep_case

pytestmark = pytest.mark.gpu

RESTART = ("phi", "fl", "T", "C", "ux", "uy", "p")
SLOW = ("phi", "fl", "T", "C")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _freezing_case():
    # a droplet on the cold wall, far enough along that a solid layer, a
    # mushy band and a flow exist
    return droplet_2d(96, 80, R=26.0, seed=7, T0=-0.05, sigma_T=-3e-4, rho_s=0.9)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_restart_from_own_fields(storage):
    import torch
    from paper_2511_09422_amd.lbfz import Solver
    cfg, phi, T, C = _freezing_case()
    a = Solver(cfg, phi, T, C, storage=storage)
    ref = Solver(cfg, phi, T, C, storage=storage)
    a.step(300)
    ref.step(300)
    f0 = a.fields(RESTART, device=True)
    assert float((1.0 - f0["fl"]).sum()) > 20.0, "no solid formed: the case does not exercise f_l"
    a.restart_fields([f0[k].contiguous() for k in RESTART])
    f1 = a.fields(RESTART)
    torch.cuda.synchronize()
    errs = {k: _rel(f1[k], f0[k].cpu().numpy()) for k in SLOW}
    print(f"[restart {storage}] re-exported fields rel L2 {errs}", flush=True)
    for k in ("phi", "fl", "C"):
        assert errs[k] <= 3e-4, (k, errs[k])
    assert errs["T"] <= 3e-3
    a.step(64)
    ref.step(64)
    fa, fr = a.fields(RESTART), ref.fields(RESTART)
    after = {k: _rel(fa[k], fr[k]) for k in RESTART}
    print(f"[restart {storage}] 64 steps on, rel L2 against the original {after}", flush=True)
    for k in SLOW:
        assert after[k] <= 1e-2, (k, after[k])
    for k in ("ux", "uy", "p"):
        assert np.isfinite(fa[k]).all()
        assert np.abs(fa[k]).max() <= 10 * np.abs(fr[k]).max() + 1e-6
    assert a.totals()["nonfinite"] == 0


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_subset_step_and_restart(storage):
    import torch
    from paper_2511_09422_amd.lbfz import Batch, LbfzError
    cases = [sweep_case(k, side=64) for k in (3, 4, 5, 6)]
    full = Batch(cases, storage=storage)
    part = Batch(cases, storage=storage)
    full.step(20)
    part.step(20)
    part.select([0, 2])
    full.step(30)
    part.step(30)
    for i in (0, 2):
        ff, fp = full.fields(i), part.fields(i)
        for k in ff:
            assert np.array_equal(ff[k], fp[k]), (i, k)
    # grids 1 and 3 were left behind: no reads, no steps
    with pytest.raises(LbfzError):
        part.fields(1)
    part.select([1])
    with pytest.raises(LbfzError):
        part.step(1)
    # restart them from the full batch's fields at this time level: grid 1
    # alone, grid 3 through the many-grid call (fields of every grid in one
    # buffer, which must agree with the per-grid reads)
    allf = torch.empty((4, 8, 64, 64), dtype=torch.float32, device="cuda")
    full.fields_all_to_device(8, allf)
    torch.cuda.synchronize()
    for i in range(4):
        fi = full.fields(i)
        for k, nm in enumerate(("phi", "fl", "T", "C", "ux", "uy", "uz", "p")):
            # the batched dry pass equals the per-grid one up to FP32 rounding
            g = allf[i, k].cpu().numpy()
            assert np.abs(g - fi[nm]).max() <= 2e-6 * max(np.abs(fi[nm]).max(), 1e-30), (i, nm)
    part.restart_fields(1, [allf[1, k] for k in range(6)] + [allf[1, 7]])
    part.restart_many([3], [allf[0, k] for k in range(6)] + [allf[0, 7]], [8 * 64 * 64] * 7)
    part.select([])
    part.step(24)
    full.step(24)
    torch.cuda.synchronize()
    for i in range(4):
        ff, fp = full.fields(i), part.fields(i)
        for k in SLOW:
            e = _rel(fp[k], ff[k])
            assert (e == 0.0) if i in (0, 2) else (e <= 1e-2), (i, k, e)
        assert part.totals(i)["nonfinite"] == 0
    full.close()
    part.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_restart_many_equals_per_grid_restarts(storage):
    """lbfz_batch_restart_many over several grids of two sizes (FP32 storage:
    one batched launch over a job table; 16-bit: per grid) leaves every grid
    in the state lbfz_batch_restart_fields gives it, bit for bit: the fields
    right after the restart and 12 steps later agree exactly; the grids not
    restarted are untouched."""
    import torch
    from paper_2511_09422_amd.lbfz import Batch
    cases = [sweep_case(k, side=64) for k in (11, 12)] + [sweep_case(k, side=128) for k in (13, 14)]
    a, b = Batch(cases, storage=storage), Batch(cases, storage=storage)
    a.step(12)
    b.step(12)
    from paper_2511_09422_amd.lbfz import RESTART_FIELDS
    n_max = 128 * 128
    # field m of grid i at R[i, m, :N_i]: grid i's own fields at this level
    # (the restart drops their non-equilibrium parts)
    R = torch.zeros((4, 7, n_max), dtype=torch.float32, device="cuda")
    for i in range(4):
        f = a.fields(i, RESTART_FIELDS)
        for m, nm in enumerate(RESTART_FIELDS):
            R[i, m, :f[nm].size] = torch.from_numpy(f[nm].reshape(-1)).cuda()
    idx = [0, 2, 3]
    a.restart_many(idx, [R[:, m] for m in range(7)], [7 * n_max] * 7)
    for i in idx:
        n = cases[i][0]["nx"] * cases[i][0]["ny"]
        b.restart_fields(i, [R[i, m, :n] for m in range(7)])
    torch.cuda.synchronize()
    for i in range(4):
        fa, fb = a.fields(i), b.fields(i)
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (storage, i, k)
    a.step(12)
    b.step(12)
    for i in range(4):
        fa, fb = a.fields(i), b.fields(i)
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (storage, i, k, "after 12 steps")
        assert a.totals(i)["nonfinite"] == 0
    a.close()
    b.close()
