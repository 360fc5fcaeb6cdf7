"""FP64 reference of the isotropic D2Q9 divergence (the stencil of the end of
Sec. 3.4 applied to u, as the phase-field source of Sec. 3.1 uses it), written
from its definition on a ghost-extended copy of the grid.  Test
infrastructure: the surrogate's screening-check kernel is compared with it."""
import numpy as np


def div_d2q9(ux, uy, walls):
    """div u by the isotropic D2Q9 stencil in FP64, from a ghost-extended copy:
    x periodic; y periodic, or no-slip walls whose ghost rows carry -u of the
    rows they mirror."""
    ux = np.asarray(ux, np.float64)
    uy = np.asarray(uy, np.float64)
    if walls:
        ex = np.concatenate([-ux[:1], ux, -ux[-1:]], 0)
        ey = np.concatenate([-uy[:1], uy, -uy[-1:]], 0)
    else:
        ex = np.concatenate([ux[-1:], ux, ux[:1]], 0)
        ey = np.concatenate([uy[-1:], uy, uy[:1]], 0)
    ny = ux.shape[0]

    def at(a, dx, dy):  # a at (x + dx, y + dy) for the rows of the grid
        return np.roll(a, -dx, axis=1)[1 + dy:ny + 1 + dy]
    dux = (at(ex, 1, 0) - at(ex, -1, 0)) / 3.0 + (at(ex, 1, 1) + at(ex, 1, -1) -
                                                  at(ex, -1, 1) - at(ex, -1, -1)) / 12.0
    duy = (at(ey, 0, 1) - at(ey, 0, -1)) / 3.0 + (at(ey, 1, 1) + at(ey, -1, 1) -
                                                  at(ey, 1, -1) - at(ey, -1, -1)) / 12.0
    return dux + duy
