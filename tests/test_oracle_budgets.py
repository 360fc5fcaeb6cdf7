"""Conservation budgets of the FP64 oracle (the paper's mass-conservation
claim, abstract and Sec. 5, with the phase-change source of Eq. NS1):

  sum_{x,i} f^{n+1} = sum f^n + sum_x phi mdot      (phase field, Sec. 3.1)
  sum_{x,i} l^{n+1} = sum l^n                       (solute, Sec. 3.4)
  sum_{x,i} h^{n+1} = sum h^n + sum_x Q             (enthalpy, adiabatic walls)

each to 1e-12 relative, on runs where the sources are substantial."""
import numpy as np
import pytest

from oracle.lbref import Oracle
from paper_2511_09422_amd.workloads import droplet_2d, droplet_3d


def _check_budgets(o, t0, norm_phi, check_h, tol=1e-12):
    t = o.totals()
    assert t["nonfinite"] == 0
    assert abs(t["sum_f"] - t0["sum_f"] - t["mpc"]) <= tol * norm_phi
    assert abs(t["sum_l"] - t0["sum_l"]) <= tol * abs(t0["sum_l"])
    if check_h:
        assert abs(t["sum_h"] - t0["sum_h"] - t["qsum"]) <= tol * max(1.0, abs(t0["sum_h"]))
    return t


def test_budgets_2d_adiabatic_with_phase_change():
    # adiabatic walls; a cold layer near the low wall freezes and the melting
    # point is off zero so that the enthalpy source Q = rho C_p T mdot is nonzero
    cfg, phi, T, C = droplet_2d(32, 32, R=11, seed=5, t_lo_dirichlet=0, T_sol=0.05,
                                T_liq=0.05, rho_s=0.8, latent=0.5, sigma_T=-4e-4)
    y = np.arange(32)[:, None] * np.ones((1, 32))
    T = T - 0.25 * np.exp(-y / 3.0)
    o = Oracle(cfg, phi, T, C)
    t0 = o.totals()
    norm = np.abs(phi).sum()
    for _ in range(10):
        o.step(20)
        t = _check_budgets(o, t0, norm, check_h=True)
    assert abs(t["mpc"]) > 1.0 and abs(t["qsum"]) > 1e-2 and t["vol_solid"] > 10


def test_budgets_2d_dirichlet_wall():
    cfg, phi, T, C = droplet_2d(32, 24, R=9, seed=6, sigma_T=-5e-4)
    o = Oracle(cfg, phi, T, C)
    t0 = o.totals()
    o.step(300)
    t = _check_budgets(o, t0, np.abs(phi).sum(), check_h=False)
    assert t["mpc"] > 0.5


def test_budgets_3d_with_obstacle():
    cfg, phi, T, C, mask = droplet_3d(16, R=7.0, imp_R=2.0, seed=1, t_lo_dirichlet=0)
    z = np.arange(16)[:, None, None]
    T = T - 0.3 * np.exp(-z / 2.0)
    o = Oracle(cfg, phi, T, C, mask=mask, threads=4)
    t0 = o.totals()
    o.step(40)
    t = _check_budgets(o, t0, np.abs(phi[mask == 0]).sum(), check_h=True)
    assert t["vol_solid"] > 5 and abs(t["mpc"]) > 0.1


def test_d3q7_fp32_weights_sum_to_one():
    """The D3Q7 weights of the FP32 evaluations (the GPU kernels' 3D
    phase-field and solute collisions and the oracle's single_cw build):
    fl(1/6) on the x and y links, (1 - 4 fl(1/6)) / 2 on the z links, which
    is one ulp below fl(1/6), every step of it exact in FP32.  The six sum to
    exactly one as reals; six fl(1/6) do not."""
    from fractions import Fraction
    hi = np.float32(1.0 / 6.0)
    lo = (np.float32(1.0) - np.float32(4.0) * hi) / np.float32(2.0)
    assert lo.dtype == np.float32 and lo == np.nextafter(hi, np.float32(0.0))
    assert lo == np.float32(0.1666666567325592)
    assert 4 * Fraction(float(hi)) + 2 * Fraction(float(lo)) == 1
    assert 6 * Fraction(float(hi)) - 1 == Fraction(1, 2 ** 25)


def test_fp32_oracle_build_with_unit_weight_sums_conserves_mass():
    """What the single_cw build is for: with weights summing to one in FP32
    its phase-field and solute masses stay with the FP64 oracle's, where the
    plain FP32 build's drift (the equilibria make mass every step).  Periodic
    24^3 drop, 400 steps: the plain build's sum f is off by 1.4e-1 and its
    sum l by 1.8e-3; the single_cw build's by 1.4e-3 and 1.8e-4."""
    from tests.test_gpu_parity3d import CASES
    cfg, phi, T, C, mask = CASES["periodic"]()
    sums = {}
    for v in (None, "single", "single_cw"):
        o = Oracle(cfg, phi, T, C, mask=mask, threads=8, variant=v)
        o.step(400)
        sums[v] = [float(o.get_pops(w).astype(np.float64).sum()) for w in (0, 3)]
    for k in range(2):
        plain = abs(sums["single"][k] - sums[None][k])
        unit = abs(sums["single_cw"][k] - sums[None][k])
        assert unit * 5.0 < plain, (k, unit, plain)
