"""Seeded synthetic workloads: parameter sets and initial fields.

This module only builds inputs (parameter dictionaries and initial phi, T, C,
obstacle-mask arrays).  It holds none of the scheme's arithmetic, and it is the
one module shared by the GPU path, the FP64 oracle, the tests and the
benchmark.  Every random draw comes from ``numpy.random.default_rng(seed)``.

Geometry (all workloads): cell-centred nodes, node j at coordinate j; when
walls are present they sit at -1/2 and n-1/2 of the last axis, the other axes
are periodic.  A droplet "sitting on the wall at a 90 degree contact angle" is a
disc (sphere) centred on the low wall, which is the equilibrium shape for a
neutral wall.

Initial profile: the equilibrium interface of the phase-field model,
phi = tanh((R - d) / (sqrt(2) eps)) (the paper's Eq. 3 with phi1 = 1,
phi2 = -1).  An "interface width" W maps to eps = W / (2 sqrt 2), since
tanh(2x/W) = tanh(x/(sqrt(2) eps)).
"""
from __future__ import annotations

import math

import numpy as np

SQRT2 = math.sqrt(2.0)


def base_params(**over) -> dict:
    """Parameters of the droplet-freezing configuration (lattice units).

    Densities rho_l = 1, rho_g = 0.1 (ratio 10), rho_s = 0.9; nu = 0.1;
    all relaxation times 0.8; interface width 4; C_p = 1 in every phase;
    T_wall = -1 (Dirichlet, low wall), high wall adiabatic; T_m = 0;
    Stefan number 1 (latent heat 1); sigma = 1e-3 - 2e-4 T; k_p = 0.5,
    D_s = D_l.  (rho C)_ref = 0.1 is the smallest phase heat capacity; with
    the D2Q5/D3Q7 enthalpy equilibrium any larger constant makes the rest
    population negative in the gas and the scheme unstable.
    """
    p = dict(
        dim=2, nx=64, ny=64, nz=1, walls=1, t_lo_dirichlet=1, t_hi_dirichlet=0,
        surface_tension_mode=0,
        rho_l=1.0, rho_g=0.1, rho_s=0.9, nu=0.1,
        tau_phi=0.8, tau_h=0.8, tau_c=0.8, eps=4.0 / (2.0 * SQRT2),
        sigma0=1e-3, sigma_T=-2e-4, sigma_c=0.0, T_ref=0.0, c_ref=0.0,
        cp_l=1.0, cp_s=1.0, cp_g=1.0, rhoc_ref=0.1,
        latent=1.0, T_sol=0.0, T_liq=0.0, k_p=0.5, Ds_over_Dl=1.0,
        T_lo=-1.0, T_hi=0.0, T_lo_amp=0.0, body_force=(0.0, 0.0, 0.0),
    )
    p.update(over)
    return p


def droplet_2d(nx: int = 64, ny: int = 64, R: float = 16.0, seed: int = 0, T0: float = 0.1,
               noise: float = 1e-3, C0: float = 0.05, **over):
    """Liquid droplet (radius R) on the cold low wall, centre (nx/2, -1/2).

    Returns (params, phi, T, C) with fields shaped (ny, nx).
    T = T0 + U(-noise, noise) from default_rng(seed); C = C0 inside the
    liquid, weighted by (1 + phi)/2 across the interface.
    """
    p = base_params(nx=nx, ny=ny, **over)
    eps = p["eps"]
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    d = np.sqrt((x - nx / 2.0) ** 2 + (y + 0.5) ** 2)
    phi = np.tanh((R - d) / (SQRT2 * eps))
    rng = np.random.default_rng(seed)
    T = T0 + rng.uniform(-noise, noise, size=(ny, nx))
    C = C0 * np.clip(0.5 * (1.0 + phi), 0.0, 1.0)
    return p, phi, T, C


def impurity_offset(seed: int = 1, scale: float = 1.0):
    """Seeded offset (dx, dy, h) of the insoluble impurity: dx, dy ~ U(-16, 16),
    height above the wall h ~ U(24, 40), all multiplied by ``scale``."""
    rng = np.random.default_rng(seed)
    dx, dy = rng.uniform(-16.0, 16.0, size=2)
    h = rng.uniform(24.0, 40.0)
    return dx * scale, dy * scale, h * scale


def droplet_3d(n: int = 256, R: float = 64.0, imp_R: float = 12.0, seed: int = 1,
               T0: float = 0.1, noise: float = 1e-3, C0: float = 0.05, **over):
    """Hemispherical droplet (radius R) on the cold low z-wall, centre
    (n/2, n/2, -1/2), holding a fixed spherical obstacle of radius imp_R at
    a seeded offset (scaled with n/256).  Returns (params, phi, T, C, mask)
    with fields shaped (n, n, n) as [z][y][x]."""
    p = base_params(dim=3, nx=n, ny=n, nz=n, **over)
    eps = p["eps"]
    dx, dy, h = impurity_offset(seed, scale=n / 256.0)
    # broadcast axes ([z][y][x]) instead of full coordinate grids
    a = np.arange(n, dtype=np.float64)
    z, y, x = a[:, None, None], a[None, :, None], a[None, None, :]
    c = n / 2.0
    d = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z + 0.5) ** 2)
    phi = np.tanh((R - d) / (SQRT2 * eps))
    di = np.sqrt((x - c - dx) ** 2 + (y - c - dy) ** 2 + (z - h) ** 2)
    mask = (di <= imp_R).astype(np.uint8)
    if mask.sum() == 0 or (h + imp_R) >= R:
        raise ValueError("impurity must lie inside the droplet")
    rng = np.random.default_rng(seed)
    T = T0 + rng.uniform(-noise, noise, size=(n, n, n))
    C = C0 * np.clip(0.5 * (1.0 + phi), 0.0, 1.0)
    return p, phi, T, C, mask


SWEEP_SIDES = (64, 128, 256, 512)


def sweep_params(k: int):
    """The draws of sweep case k: (side, Marangoni coefficient, Stefan number,
    rho_s / rho_l, C0), from default_rng(1000 + k) in that order."""
    rng = np.random.default_rng(1000 + k)
    side = int(rng.choice(SWEEP_SIDES))
    coef = float(rng.uniform(0.0, 5e-4))
    ste = float(rng.uniform(0.5, 2.0))
    rr = float(rng.uniform(0.85, 1.0))
    c0 = float(rng.uniform(0.0, 0.1))
    return side, coef, ste, rr, c0


def sweep_case(k: int, side: int = 0, **over):
    """Case k of the parameter sweep: default_rng(1000 + k) draws, in order,
    the side in {64, 128, 256, 512}, the Marangoni coefficient in [0, 5e-4]
    (sigma_T = -coefficient), the Stefan number in [0.5, 2], the solid/liquid
    density ratio in [0.85, 1.0] and the initial solute C0 in [0, 0.1]; the
    droplet radius is side/4.  side != 0 keeps the other draws and replaces
    the side (the surrogate's training and held-out grids).  Returns
    (params, phi, T, C)."""
    s, coef, ste, rr, c0 = sweep_params(k)
    side = side or s
    p, phi, T, C = droplet_2d(side, side, R=side / 4.0, seed=1000 + k, C0=c0,
                              sigma_T=-coef, latent=1.0 / ste, rho_s=rr, **over)
    p["case"] = k
    p["stefan"] = ste
    return p, phi, T, C
