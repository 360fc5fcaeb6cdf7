"""The C oracle's 3D step against an independent naive evaluator (pure
Python, mpmath at 40 digits, per node and per direction) for one and two
steps on a 5 x 4 x 6 grid with walls on z and a one-node obstacle, from
seeded random states that exercise every term: phase change in progress,
non-equilibrium populations, nonzero previous velocity / pressure / phi / C,
both wall kinds, the D3Q19 edge links that cross a wall, and every obstacle
rule (stencil values, velocity ghost, bounce-back of f, g, l, conduction of
h)."""
import numpy as np
import pytest
from mpmath import mpf

from oracle.lbref import Oracle
from paper_2511_09422_amd.workloads import base_params
from tests import bruteforce_step3d as bf

NX, NY, NZ = 5, 4, 6
OBST = (3, 1, 2)        # (z, y, x) of the obstacle node
W7 = np.array([0.0] + [1 / 6] * 6)


def _random_state(seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(NZ, dtype=float), np.arange(NY, dtype=float),
                          np.arange(NX, dtype=float), indexing="ij")
    d = np.sqrt((x - NX / 2 + 0.3) ** 2 + (y - NY / 2 + 0.2) ** 2 + (z + 0.5) ** 2)
    phi = np.tanh((3.6 - d) / 2.0)
    mask = np.zeros((NZ, NY, NX), np.uint8)
    mask[OBST] = 1
    f = W7[:, None, None, None] * phi * (1 + 0.02 * rng.normal(size=(7, NZ, NY, NX)))
    f[0] = 0.02 * rng.normal(size=(NZ, NY, NX)) * (1 + phi) / 2
    T = 0.02 * rng.normal(size=(NZ, NY, NX)) - 0.01 * z / NZ
    psi = np.clip((1 + phi) / 2, 0, 1)
    E = (psi * 1.0 + (1 - psi) * 0.1) * T + psi * 1.0 * (0.3 + 0.6 * rng.uniform(size=T.shape))
    h = np.empty((7, NZ, NY, NX))
    h[1:] = (1 / 6) * 0.1 * T * (1 + 0.05 * rng.normal(size=(6, NZ, NY, NX)))
    h[0] = E - h[1:].sum(0)
    g = 1e-4 * rng.normal(size=(19, NZ, NY, NX))
    Cc = 0.05 * psi
    l = W7[:, None, None, None] * Cc * (1 + 0.03 * rng.normal(size=(7, NZ, NY, NX)))
    l[0] = 1e-3 * rng.normal(size=(NZ, NY, NX)) * psi
    state = dict(fs=0.3 * psi * rng.uniform(size=T.shape), p=1e-4 * rng.normal(size=T.shape),
                 ux=1e-3 * rng.normal(size=T.shape), uy=1e-3 * rng.normal(size=T.shape),
                 uz=1e-3 * rng.normal(size=T.shape),
                 phi=phi + 0.01 * rng.normal(size=T.shape), C=Cc + 1e-3 * rng.normal(size=T.shape))
    # the obstacle node carries what the scheme keeps there: no phase field,
    # solute, flow or solid; its enthalpy is free
    for k in ("f", "g", "l"):
        arr = dict(f=f, g=g, l=l)[k]
        arr[(slice(None),) + OBST] = 0.0
    for k in ("fs", "p", "ux", "uy", "uz", "C"):
        state[k][OBST] = 0.0
    state["phi"][OBST] = -1.0
    return phi, mask, dict(f=f, g=g, h=h, l=l), state


def _to_mp(a):
    if a.ndim == 1:
        return [mpf(float(v)) for v in a]
    return [_to_mp(s) for s in a]


def _to_np(a):
    if isinstance(a[0], list):
        return np.array([_to_np(s) for s in a])
    return np.array([float(v) for v in a])


STATE_SLOTS = (("fs", 0), ("p", 1), ("ux", 2), ("uy", 3), ("uz", 4), ("phi", 5), ("C", 6))


@pytest.mark.parametrize("seed,over", [
    (21, dict()),
    (22, dict(t_hi_dirichlet=1, T_hi=0.2, T_lo_amp=0.3, sigma_c=-3e-3, Ds_over_Dl=0.3,
              T_sol=-0.05, T_liq=0.04, rho_s=0.85, surface_tension_mode=1,
              body_force=(1e-6, -2e-6, 3e-6))),
])
def test_oracle_3d_matches_naive_evaluator(seed, over):
    cfg = base_params(dim=3, nx=NX, ny=NY, nz=NZ, sigma_T=-3e-3, **over)
    phi, mask, pops, state = _random_state(seed)
    o = Oracle(cfg, phi, np.zeros_like(phi), np.zeros_like(phi), mask=mask)
    for k, w in (("f", 0), ("g", 1), ("h", 2), ("l", 3)):
        o.set_pops(w, pops[k])
    for k, w in STATE_SLOTS:
        o.set_state(w, state[k])
    Pm = dict(cfg)
    Pm["body_force"] = [mpf(v) for v in cfg["body_force"]]
    mp_pops = {k: _to_mp(v) for k, v in pops.items()}
    mp_state = {k: _to_mp(v) for k, v in state.items()}
    mmask = mask.tolist()
    for nstep in (1, 2):
        mp_pops, mp_state = bf.step(Pm, mp_pops, mp_state, mmask)
        o.step(1)
        for k, w in (("f", 0), ("g", 1), ("h", 2), ("l", 3)):
            ref = _to_np(mp_pops[k])
            got = o.get_pops(w)
            scale = np.abs(ref).max()
            assert np.abs(got - ref).max() <= 1e-12 * scale, (nstep, k, np.abs(got - ref).max(),
                                                              scale)
        for k, w in STATE_SLOTS:
            ref = _to_np(mp_state[k])
            got = o.get_state(w)
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(got - ref).max() <= 1e-11 * scale, (nstep, k)
    # the random state exercises phase change, the solid drag and flow next
    # to the obstacle and the walls
    assert np.asarray(o.get_state(0)).max() > 0.05
    u = np.asarray(o.get_state(2))
    assert np.abs(u[0]).max() > 1e-5 and np.abs(u[OBST[0] - 1]).max() > 1e-5
