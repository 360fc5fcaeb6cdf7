"""The column-window method of the full-size 3D parity test, checked on the
oracle alone: one step of a 16 x 16 x nz window of a state, stepped on its
own with periodic x and y, equals the whole grid's step in the window's core
(four nodes from its edge) bit for bit, and differs at the edge."""
import os

import numpy as np

from oracle.lbref import Oracle
from paper_2511_09422_amd.workloads import droplet_3d

THREADS = min(8, os.cpu_count() or 1)
FIELDS = ("phi", "fl", "T", "C", "ux", "uy", "uz", "p")


def _window(a, x0, y0, w):
    nx, ny = a.shape[-1], a.shape[-2]
    xs = np.arange(x0, x0 + w) % nx
    ys = np.arange(y0, y0 + w) % ny
    return np.take(np.take(a, ys, axis=-2), xs, axis=-1)


def _state(o):
    return np.concatenate([o.get_pops(0), o.get_pops(1), o.get_pops(2), o.get_pops(3)] +
                          [o.get_state(w)[None] for w in range(7)])


def _from_state(cfg, st, shape, mask):
    z = np.zeros(shape)
    o = Oracle(cfg, z, z, z, mask=mask, threads=THREADS)
    for which, sl in ((0, slice(0, 7)), (1, slice(7, 26)), (2, slice(26, 33)),
                      (3, slice(33, 40))):
        o.set_pops(which, st[sl])
    for w in range(7):
        o.set_state(w, st[40 + w])
    return o


def test_window_step_equals_whole_grid_step_in_the_core():
    n, W, M = 32, 16, 4
    cfg, phi, T, C, mask = droplet_3d(n, R=9.0, imp_R=2.0, seed=1)
    o = Oracle(cfg, phi, T, C, mask=mask, threads=THREADS)
    o.step(10)
    st = _state(o)
    o.step(1)
    full = o.fields()
    core = (slice(None), slice(M, W - M), slice(M, W - M))
    edge_diff = 0.0
    for x0, y0 in ((6, 6), (-4, 20), (20, 9)):
        wcfg = dict(cfg, nx=W, ny=W)
        wm = np.ascontiguousarray(_window(mask, x0, y0, W))
        ow = _from_state(wcfg, _window(st, x0, y0, W), (n, W, W), wm)
        ow.step(1)
        r = ow.fields()
        for k in FIELDS:
            assert np.array_equal(_window(full[k], x0, y0, W)[core], r[k][core]), (x0, y0, k)
        edge_diff = max(edge_diff, float(np.abs(_window(full["phi"], x0, y0, W) - r["phi"]).max()))
    assert edge_diff > 1e-6  # the periodic wrap of a window is wrong at its edge
