"""The C oracle against an independent naive evaluator (pure Python,
mpmath at 40 digits, per node and per direction) for one and two steps on
8x8 grids from seeded random states that exercise every term of the step:
phase change in progress, non-equilibrium populations, nonzero previous
velocity / pressure / phi / C, both wall types."""
import numpy as np
import pytest
from mpmath import mpf

from oracle.lbref import Oracle
from paper_2511_09422_amd.workloads import base_params
from tests import bruteforce_step as bf

W5 = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])


def _random_state(seed, nx=8, ny=8):
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    d = np.hypot(x - nx / 2 + 0.3, y + 0.5)
    phi = np.tanh((4.5 - d) / 2.0)
    f = W5[:, None, None] * phi * (1 + 0.02 * rng.normal(size=(5, ny, nx)))
    T = 0.02 * rng.normal(size=(ny, nx)) - 0.01 * y / ny
    psi = np.clip((1 + phi) / 2, 0, 1)
    E = (psi * 1.0 + (1 - psi) * 0.1) * T + psi * 1.0 * (0.3 + 0.6 * rng.uniform(size=(ny, nx)))
    h = np.empty((5, ny, nx))
    h[1:] = W5[1:, None, None] * 0.1 * T * (1 + 0.05 * rng.normal(size=(4, ny, nx)))
    h[0] = E - h[1:].sum(0)
    g = 1e-4 * rng.normal(size=(9, ny, nx))
    Cc = 0.05 * psi
    l = W5[:, None, None] * Cc * (1 + 0.03 * rng.normal(size=(5, ny, nx)))
    state = dict(fs=0.3 * psi * rng.uniform(size=(ny, nx)), p=1e-4 * rng.normal(size=(ny, nx)),
                 ux=1e-3 * rng.normal(size=(ny, nx)), uy=1e-3 * rng.normal(size=(ny, nx)),
                 phi=phi + 0.01 * rng.normal(size=(ny, nx)), C=Cc + 1e-3 * rng.normal(size=(ny, nx)))
    return phi, dict(f=f, g=g, h=h, l=l), state


def _to_mp(a):
    if a.ndim == 2:
        return [[mpf(float(v)) for v in row] for row in a]
    return [_to_mp(s) for s in a]


@pytest.mark.parametrize("seed,over", [
    (11, dict()),
    (12, dict(t_hi_dirichlet=1, T_hi=0.2, T_lo_amp=0.3, sigma_c=-3e-3, Ds_over_Dl=0.3,
              T_sol=-0.05, T_liq=0.04, rho_s=0.85, surface_tension_mode=1,
              body_force=(1e-6, -2e-6, 0.0))),
])
def test_oracle_matches_naive_evaluator(seed, over):
    cfg = base_params(nx=8, ny=8, sigma_T=-3e-3, **over)
    phi, pops, state = _random_state(seed)
    o = Oracle(cfg, phi, np.zeros_like(phi), np.zeros_like(phi))
    for k, w in (("f", 0), ("g", 1), ("h", 2), ("l", 3)):
        o.set_pops(w, pops[k])
    for k, w in (("fs", 0), ("p", 1), ("ux", 2), ("uy", 3), ("phi", 5), ("C", 6)):
        o.set_state(w, state[k])
    o.set_state(4, np.zeros_like(phi))
    Pm = dict(cfg)
    Pm["body_force"] = [mpf(v) for v in cfg["body_force"]]
    mp_pops = {k: _to_mp(v) for k, v in pops.items()}
    mp_state = {k: _to_mp(v) for k, v in state.items()}
    for nstep in (1, 2):
        mp_pops, mp_state = bf.step(Pm, mp_pops, mp_state)
        o.step(1)
        for k, w in (("f", 0), ("g", 1), ("h", 2), ("l", 3)):
            ref = np.array([[[float(v) for v in row] for row in q] for q in mp_pops[k]])
            got = o.get_pops(w)
            scale = np.abs(ref).max()
            assert np.abs(got - ref).max() <= 1e-12 * scale, (nstep, k, np.abs(got - ref).max(), scale)
        for k, w in (("fs", 0), ("p", 1), ("ux", 2), ("uy", 3), ("phi", 5), ("C", 6)):
            ref = np.array([[float(v) for v in row] for row in mp_state[k]])
            got = o.get_state(w)
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(got - ref).max() <= 1e-11 * scale, (nstep, k)
    # the random state does exercise phase change and the solid drag
    assert np.asarray(o.get_state(0)).max() > 0.05
