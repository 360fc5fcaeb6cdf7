"""Host logic of the surrogate screening check, on synthetic sums (no GPU).

Each LB step adds sum phi div u to sum phi (the phase-field source of Sec.
3.1, which carries both the volume change of freezing, div u = mdot of Eq.
NS1, and the flow's compression), so over a stride of STRIDE steps the
check's residual is
    |sum phi_after - sum phi_before - (STRIDE / 2)(q_before + q_after)|
over the liquid volume sum (1 + phi_before) / 2, with q = sum phi div u of
either end (the trapezoid rule).  Optionally the solute drift (the solute
budget of Sec. 3.4 is exact) is checked too; a prediction is accepted when
they stay within their tolerances and it is finite."""
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


def test_a_change_that_follows_the_budget_has_zero_residual():
    """sum phi moves by exactly STRIDE times the mean of the two ends' sum
    phi div u: residual zero, accepted, whatever happened to f_l."""
    b = _droplet()
    n = b[0].size
    q_b, q_a = 0.37, 0.21                       # sum phi div u at either end
    a = [f.copy() for f in b]
    idx = np.argwhere(b[0] > 0.99)[:37]
    a[1][tuple(idx.T)] = 0.0                    # 37 nodes freeze
    a[0] = a[0] + 0.5 * sg.STRIDE * (q_b + q_a) / n
    ok, r, d = sg.check(_sums(b), _sums(a), n, q_b, q_a)
    assert ok and r < 1e-12 and d == 0.0


def test_residual_sign_and_scale():
    """A state that does not move while its ends report a divergence: the
    residual is the budget's stride integral over the liquid volume, the same
    magnitude for the reversed pair with the divergences negated."""
    b = _droplet(seed=1)
    n = b[0].size
    liquid = 0.5 * (n + b[0].sum())
    q_b, q_a = 1e-3, 3e-3
    _, r, _ = sg.check(_sums(b), _sums(b), n, q_b, q_a)
    assert abs(r - 0.5 * sg.STRIDE * (q_b + q_a) / liquid) < 1e-15
    a = [f.copy() for f in b]
    a[0] = a[0] + 0.5 * sg.STRIDE * (q_b + q_a) / n
    _, r_fwd, _ = sg.check(_sums(b), _sums(a), n, 0.0, 0.0)
    _, r_back, _ = sg.check(_sums(a), _sums(b), n, 0.0, 0.0)
    assert abs(r_fwd - r) < 1e-12
    assert abs(r_back - 0.5 * sg.STRIDE * (q_b + q_a) / (0.5 * (n + a[0].sum()))) < 1e-12


def test_threshold_on_phi_mass():
    b = _droplet(seed=2)
    n = b[0].size
    liquid = 0.5 * (n + b[0].sum())
    for excess, want in ((0.5e-3, True), (2e-3, False)):
        a = [f.copy() for f in b]
        a[0] = a[0] + excess * liquid / n   # uniform phi drift: sum dphi = excess * liquid
        ok, r, _ = sg.check(_sums(b), _sums(a), n, 0.0, 0.0)
        assert abs(r - excess) < 1e-9 and ok is want


def test_solute_drift_and_non_finite_predictions():
    b = _droplet(seed=3)
    n = b[0].size
    a = [f.copy() for f in b]
    a[3] = a[3] * (1 + 1e-3)                # sum C drifts by 1e-3
    ok, r, d = sg.check(_sums(b), _sums(a), n, 0.0, 0.0, solute_tol=None)
    assert ok and r == 0.0 and abs(d - 1e-3) < 1e-9   # phi mass only
    assert not sg.check(_sums(b), _sums(a), n, 0.0, 0.0, solute_tol=5e-4)[0]
    a[3] = b[3] * (1 + 2e-3)                # the default tolerance is 1e-3
    assert not sg.check(_sums(b), _sums(a), n, 0.0, 0.0)[0]
    a[3] = b[3].copy()
    a[3][0, 0] += 1e-4 * b[3].sum()        # 1e-4 < 5e-4: accepted
    assert sg.check(_sums(b), _sums(a), n, 0.0, 0.0, solute_tol=5e-4)[0]
    a[0] = a[0].copy()
    a[0][5, 5] = np.nan
    assert not sg.check(_sums(b), _sums(a), n, 0.0, 0.0, solute_tol=None)[0]
    # a non-finite predicted velocity shows in its sum phi div u
    assert not sg.check(_sums(b), _sums(b), n, 0.0, np.inf)[0]


def test_check_all_equals_check_per_grid():
    """The vectorised check over many grids returns exactly what check()
    returns grid by grid: random sums around the accept threshold, a
    non-finite prediction, a non-finite divergence sum, a zero solute sum,
    with and without the solute tolerance."""
    rng = np.random.default_rng(3)
    n, npx = 40, 256 * 256
    sb = rng.uniform(-1, 1, size=(n, 8)) * npx * np.array([0.3, 1, 0.1, 0.05, 1e-3, 1e-3, 0, 1e-4])
    sa = sb + rng.normal(0, 1, size=(n, 8)) * np.array([30, 10, 1, 1e-3, 1e-4, 1e-4, 0, 1e-5])
    qb = rng.normal(0, 0.3, size=n)
    qa = qb + rng.normal(0, 0.2, size=n)
    sa[5, 2] = np.nan
    qa[9] = np.nan
    sb[7, 3] = 0.0
    for tol in (None, 1e-4):
        got = sg.check_all(sb, sa, npx, qb, qa, sg.MASS_TOL, tol)
        ref = [sg.check(sb[i], sa[i], npx, qb[i], qa[i], sg.MASS_TOL, tol) for i in range(n)]
        assert [g[0] for g in got] == [r[0] for r in ref]
        # equal values, a NaN residual (grid 9) included
        np.testing.assert_array_equal(np.array([g[1:] for g in got]),
                                      np.array([r[1:] for r in ref]))
    assert 0 < sum(g[0] for g in got) < n and not got[5][0] and not got[9][0]
