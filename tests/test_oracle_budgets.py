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
