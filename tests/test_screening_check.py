"""Host logic of the surrogate screening check, on synthetic fields (no GPU):
the phase-field mass residual |sum dphi - (1 - rho_s/rho_l) sum df_s| /
sum (1 + phi)/2 (freezing changes the volume by the density ratio, Eq. NS1)
and, optionally, the solute drift (the solute budget of Sec. 3.4 is exact);
a prediction is accepted when they stay within their tolerances and it is
finite."""
import numpy as np

from paper_2511_09422_amd import surrogate as sg


def _sums(fields):
    return np.array([f.astype(np.float64).sum() for f in fields])


def _droplet(n=64, seed=0):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:n, 0:n]
    phi = np.tanh((n / 4 - np.hypot(x - n / 2, y - n / 3)) / 2.0)
    fl = np.ones((n, n))                       # nothing frozen yet
    T = 0.1 * rng.standard_normal((n, n))
    C = 0.05 * (1 + phi) + 0.01 * rng.random((n, n))
    return [phi, fl, T, C]


def test_freezing_with_the_density_ratio_has_zero_residual():
    b = _droplet()
    ratio = 1.0 - 0.9 / 1.0
    a = [f.copy() for f in b]
    # 37 liquid nodes freeze (f_l 1 -> 0, sum df_s = 37) and phi grows by
    # ratio at each of them: sum dphi = ratio * sum df_s
    idx = np.argwhere(b[0] > 0.99)[:37]
    assert len(idx) == 37
    a[1][tuple(idx.T)] = 0.0
    a[0][tuple(idx.T)] += ratio
    n = b[0].size
    ok, r, d = sg.check(_sums(b), _sums(a), n, ratio)
    assert ok and r < 1e-12 and d == 0.0


def test_residual_sign_and_scale():
    b = _droplet(seed=1)
    ratio = 0.12
    n = b[0].size
    liquid = 0.5 * (n + b[0].sum())
    a = [f.copy() for f in b]
    a[1][:4, :4] = 0.0                     # 16 nodes freeze (df_s = +16)...
    # ... but phi does not move: residual = ratio * 16 / liquid volume
    _, r, _ = sg.check(_sums(b), _sums(a), n, ratio)
    assert abs(r - ratio * 16 / liquid) < 1e-12
    # melting the same nodes the other way gives the same magnitude
    _, r2, _ = sg.check(_sums(a), _sums(b), n, ratio)
    assert abs(r2 - r) < 1e-9


def test_threshold_on_phi_mass():
    b = _droplet(seed=2)
    n = b[0].size
    liquid = 0.5 * (n + b[0].sum())
    for excess, want in ((0.5e-3, True), (2e-3, False)):
        a = [f.copy() for f in b]
        a[0] = a[0] + excess * liquid / n   # uniform phi drift: sum dphi = excess * liquid
        ok, r, _ = sg.check(_sums(b), _sums(a), n, 0.1)
        assert abs(r - excess) < 1e-9 and ok is want


def test_solute_drift_and_non_finite_predictions():
    b = _droplet(seed=3)
    n = b[0].size
    a = [f.copy() for f in b]
    a[3] = a[3] * (1 + 1e-3)                # sum C drifts by 1e-3
    ok, r, d = sg.check(_sums(b), _sums(a), n, 0.1)
    assert ok and r == 0.0 and abs(d - 1e-3) < 1e-9   # the default checks phi mass only
    assert not sg.check(_sums(b), _sums(a), n, 0.1, solute_tol=5e-4)[0]
    a[3] = b[3].copy()
    a[3][0, 0] += 1e-4 * b[3].sum()        # 1e-4 < 5e-4: accepted
    assert sg.check(_sums(b), _sums(a), n, 0.1, solute_tol=5e-4)[0]
    a[0] = a[0].copy()
    a[0][5, 5] = np.nan
    assert not sg.check(_sums(b), _sums(a), n, 0.1)[0]


def test_check_all_equals_check_per_grid():
    """The vectorised check over many grids returns exactly what check()
    returns grid by grid: random sums around the accept threshold, a
    non-finite prediction, a zero solute sum, with and without the solute
    tolerance."""
    rng = np.random.default_rng(3)
    n, npx = 40, 256 * 256
    sb = rng.uniform(-1, 1, size=(n, 8)) * npx * np.array([0.3, 1, 0.1, 0.05, 1e-3, 1e-3, 1, 1])
    sa = sb[:, :6] + rng.normal(0, 1, size=(n, 6)) * np.array([30, 10, 1, 1e-3, 1e-4, 1e-4])
    sa[5, 2] = np.nan
    sb[7, 3] = 0.0
    ratios = rng.uniform(0, 0.15, size=n)
    for tol in (None, 1e-4):
        got = sg.check_all(sb, sa, npx, ratios, sg.MASS_TOL, tol)
        ref = [sg.check(sb[i], sa[i], npx, ratios[i], sg.MASS_TOL, tol) for i in range(n)]
        assert got == ref
    assert 0 < sum(g[0] for g in got) < n and not got[5][0]
