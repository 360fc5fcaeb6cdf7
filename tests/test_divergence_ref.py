"""Pins of the FP64 divergence reference (tests/divergence_ref.py) against
closed forms: the surrogate screening kernel's GPU test relies on it."""
import numpy as np

from tests.divergence_ref import div_d2q9


def test_divergence_reference_closed_forms():
    """The reference stencil itself: on a periodic grid the isotropic D2Q9
    divergence of (sin kx, sin ly) is sin k cos kx + sin l cos ly exactly; at
    no-slip walls a flow parallel to them that is uniform in y has no
    divergence, and a wall-normal flow that is uniform in x has the
    one-sided difference of the mirrored ghost."""
    nx, ny = 48, 40
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    k, l = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    d = div_d2q9(np.sin(k * x), np.sin(l * y), walls=0)
    assert np.abs(d - (np.sin(k) * np.cos(k * x) + np.sin(l) * np.cos(l * y))).max() < 1e-13
    assert np.abs(div_d2q9(np.sin(k * x) * 0 + 1.0, np.zeros((ny, nx)), walls=1)).max() < 1e-15
    v = np.ones((ny, nx))
    d = div_d2q9(np.zeros((ny, nx)), v, walls=1)
    # interior rows: zero; row 0: (v - (-v)) / 3 + 2 (v - (-v)) / 12 = v; last row: -v
    assert np.abs(d[1:-1]).max() == 0.0
    assert np.allclose(d[0], 1.0) and np.allclose(d[-1], -1.0)
