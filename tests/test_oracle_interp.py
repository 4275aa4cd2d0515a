"""Pins of the oracle's mixed-order atmosphere interpolator (Sect. 4,
strategy (d)) and of the synthetic table it is fed.

* node reproduction: at every table node the interpolant returns the node;
* polynomial exactness: a table that is linear in logT and log g and cubic
  in mu and x is reproduced exactly inside the cubic zones; in the protected
  small-mu zone (the four smallest-mu nodes) and the last mu interval the
  result is the linear interpolant of the two bracketing nodes; in the
  first and last x interval it is linear as well;
* outside the x axis the intensity is zero; logT and log g are clamped;
* strategy (a) (cubic on all four axes, stencils shifted inward at the
  axis ends) reproduces a table cubic in every axis exactly, edge intervals
  included, where (d) does not; strategy (c) is (a) but linear in the
  protected zone; strategy (b) is max(0, (a)), and on a steep limb (a)
  undershoots below zero in the small-mu intervals while (c) and (d) do not;
* the synthetic table is blackbody x cubic limb polynomial: the interpolant
  is exact in mu, logT and log g away from the linear zones and within the
  cubic Lagrange remainder bound in x.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as syn


def table_spec(logi, axes):
    return dict(mode=1, intensity=1, n_spots=1, shape=[0, 0], n_rings=[1, 1], n_phi=[1, 1],
                shape_a=[0, 0], shape_b=[0, 0], n_fp=4, n_phase=1, energy=np.ones(1), t_exp=1.0,
                sigma=None, rsp=np.ones((1, 1)), atmos_logI=logi, atmos_axes=axes)


AX = syn.atmosphere_axes()


def poly_table(fn):
    at, ag, am, ax = AX
    T, G, M, X = np.meshgrid(at, ag, am, ax, indexing="ij")
    lin = fn(T, G, M, X)
    return lin


def make(fn):
    lin = poly_table(fn)
    # the oracle reads log10 values; positive tables only
    return table_spec(np.log10(lin), AX), lin


def cubic_fn(T, G, M, X):
    return (3.0 + 0.5 * (T - 6) + 0.3 * (G - 14.2)) * (2 + M - 0.7 * M ** 2 + 0.4 * M ** 3) * \
        (5 + X + 0.3 * X ** 2 - 0.2 * X ** 3)


def test_node_reproduction():
    spec, lin = make(cubic_fn)
    at, ag, am, ax = AX
    rng = np.random.default_rng(0)
    for _ in range(300):
        a, b, c, d = (rng.integers(0, len(v)) for v in AX)
        v = oracle.atmo(spec, lin, at[a], ag[b], am[c], ax[d])
        assert v == pytest.approx(lin[a, b, c, d], rel=1e-13)


def test_polynomial_exactness_and_linear_zones():
    spec, lin = make(cubic_fn)
    at, ag, am, ax = AX
    rng = np.random.default_rng(1)
    for _ in range(400):
        lt = rng.uniform(at[0], at[-1])
        lg = rng.uniform(ag[0], ag[-1])
        x = rng.uniform(ax[1], ax[-2])          # inside the cubic x zone
        m = rng.uniform(am[3], am[-2])          # inside the cubic mu zone
        exact = cubic_fn(lt, lg, m, x)
        assert oracle.atmo(spec, lin, lt, lg, m, x) == pytest.approx(exact, rel=1e-12)
    # protected mu zone: linear between the bracketing nodes
    for k in range(3):
        m = am[k] + 0.37 * (am[k + 1] - am[k])
        lt, lg, x = 6.03, 14.33, 0.41
        f0 = cubic_fn(lt, lg, am[k], x)
        f1 = cubic_fn(lt, lg, am[k + 1], x)
        want = f0 + 0.37 * (f1 - f0)
        assert oracle.atmo(spec, lin, lt, lg, m, x) == pytest.approx(want, rel=1e-12)
        # and strategy (a) (cubic) is different there (for k >= 1)
        if k >= 1:
            assert abs(oracle.atmo(spec, lin, lt, lg, m, x, mode=1) / want - 1) > 1e-8
    # last mu interval: linear
    m = am[-2] + 0.6 * (am[-1] - am[-2])
    f0, f1 = cubic_fn(6.0, 14.2, am[-2], 0.3), cubic_fn(6.0, 14.2, am[-1], 0.3)
    assert oracle.atmo(spec, lin, 6.0, 14.2, m, 0.3) == pytest.approx(f0 + 0.6 * (f1 - f0), rel=1e-12)
    # first / last x interval: linear
    for x0, x1, t in ((ax[0], ax[1], 0.3), (ax[-2], ax[-1], 0.8)):
        x = x0 + t * (x1 - x0)
        f0, f1 = cubic_fn(6.0, 14.2, 0.5, x0), cubic_fn(6.0, 14.2, 0.5, x1)
        assert oracle.atmo(spec, lin, 6.0, 14.2, 0.5, x) == pytest.approx(f0 + t * (f1 - f0), rel=1e-12)


def test_ranges():
    spec, lin = make(cubic_fn)
    at, ag, am, ax = AX
    assert oracle.atmo(spec, lin, 6.0, 14.2, 0.5, ax[0] - 1e-9) == 0.0
    assert oracle.atmo(spec, lin, 6.0, 14.2, 0.5, ax[-1] + 1e-9) == 0.0
    # clamps
    assert oracle.atmo(spec, lin, at[-1] + 0.3, 14.2, 0.5, 0.1) == pytest.approx(
        oracle.atmo(spec, lin, at[-1], 14.2, 0.5, 0.1), rel=1e-15)
    assert oracle.atmo(spec, lin, 6.0, ag[0] - 0.2, 0.5, 0.1) == pytest.approx(
        oracle.atmo(spec, lin, 6.0, ag[0], 0.5, 0.1), rel=1e-15)
    assert oracle.atmo(spec, lin, 6.0, 14.2, 0.0, 0.1) == pytest.approx(
        oracle.atmo(spec, lin, 6.0, 14.2, am[0], 0.1), rel=1e-15)


def lagrange_remainder_bound(f4max, x, nodes):
    return f4max / 24.0 * abs(np.prod(x - nodes))


def test_synthetic_table_closed_form():
    logi, axes = syn.atmosphere_table()
    at, ag, am, ax = axes
    spec = table_spec(logi, axes)
    lin = 10.0 ** logi
    a0, aT, ag_ = syn.limb_polynomial_coeffs()
    pref = 2 * syn.K_B_KEV ** 3 / (syn.H_KEVS ** 3 * syn.C_CGS ** 2)

    def V(lt, lg, m, x):
        y = 10.0 ** x
        a = a0 + aT * (lt - 6) + ag_ * (lg - 14.2)
        return pref * y ** 3 / math.expm1(y) * (1 + a[0] * m + a[1] * m * m + a[2] * m ** 3)

    h = ax[1] - ax[0]

    def bb(x):
        y = 10.0 ** x
        return pref * y ** 3 / np.expm1(y)

    rng = np.random.default_rng(3)
    for _ in range(300):
        lt = rng.uniform(at[0], at[-1])
        lg = rng.uniform(ag[0], ag[-1])
        m = rng.uniform(am[3], am[-2])
        j = int(rng.integers(1, len(ax) - 2))
        # exact at x nodes (the mu, logT, log g directions are reproduced exactly)
        assert oracle.atmo(spec, lin, lt, lg, m, ax[j]) == pytest.approx(V(lt, lg, m, ax[j]), rel=1e-12)
        # inside interval j: P(mu) times the cubic Lagrange error of the
        # blackbody factor, bounded by max|d4 bb| / 24 * |prod(x - x_i)|
        xj = ax[j] + rng.uniform(0.05, 0.95) * h
        nodes = ax[j - 1:j + 3]
        xs = np.linspace(nodes[0], nodes[-1], 4001)
        d4 = np.abs(np.diff(bb(xs), 4)).max() / (xs[1] - xs[0]) ** 4
        pm = V(lt, lg, m, xj) / bb(xj)
        bound = 1.1 * d4 / 24.0 * abs(np.prod(xj - nodes)) * pm
        err = abs(oracle.atmo(spec, lin, lt, lg, m, xj) - V(lt, lg, m, xj))
        assert err <= bound + 1e-12 * V(lt, lg, m, xj)


# ---------------------------------------------------------------- strategies (a)-(c)
def cubic4_fn(T, G, M, X):
    """Cubic in each of the four axes (logT and log g included)."""
    t, g = T - 6.0, G - 14.2
    return (3.0 + 0.5 * t - 0.8 * t ** 2 + 0.6 * t ** 3) * (2.0 + 0.3 * g + 0.9 * g ** 2 - 0.7 * g ** 3) * \
        (2 + M - 0.7 * M ** 2 + 0.4 * M ** 3) * (5 + X + 0.3 * X ** 2 - 0.2 * X ** 3)


def test_strategy_a_cubic_everywhere_is_exact_for_cubics():
    """Strategy (a): four-node Lagrange on every axis, stencils shifted inward
    at the axis ends, so a table cubic in each axis is reproduced exactly
    everywhere inside the axes, edge intervals included; the mixed default
    (d) is not (linear in logT and log g)."""
    spec, lin = make(cubic4_fn)
    at, ag, am, ax = AX
    rng = np.random.default_rng(7)
    worst_d = 0.0
    for _ in range(300):
        lt = rng.uniform(at[0], at[-1])
        lg = rng.uniform(ag[0], ag[-1])
        m = rng.uniform(am[0], am[-1])
        x = rng.uniform(ax[0], ax[-1])
        exact = cubic4_fn(lt, lg, m, x)
        assert oracle.atmo(spec, lin, lt, lg, m, x, mode=1) == pytest.approx(exact, rel=1e-11)
        worst_d = max(worst_d, abs(oracle.atmo(spec, lin, lt, lg, m, x, mode=0) / exact - 1))
    assert worst_d > 1e-6
    # edge intervals of every axis
    for lt, lg, m, x in ((at[0] + 0.3 * (at[1] - at[0]), ag[-1] - 0.2 * (ag[-1] - ag[-2]),
                          am[0] + 0.5 * (am[1] - am[0]), ax[0] + 0.4 * (ax[1] - ax[0])),
                         (at[-1] - 0.1 * (at[-1] - at[-2]), ag[0] + 0.7 * (ag[1] - ag[0]),
                          am[-1] - 0.3 * (am[-1] - am[-2]), ax[-1] - 0.6 * (ax[-1] - ax[-2]))):
        assert oracle.atmo(spec, lin, lt, lg, m, x, mode=1) == pytest.approx(cubic4_fn(lt, lg, m, x), rel=1e-11)


def test_strategy_c_linear_only_in_protected_zone():
    """Strategy (c): as (a) except linear in mu between the bracketing nodes
    in the three smallest-mu intervals."""
    spec, lin = make(cubic4_fn)
    at, ag, am, ax = AX
    lt, lg, x = 6.37, 14.03, 0.77
    for k in range(3):
        m = am[k] + 0.41 * (am[k + 1] - am[k])
        f0 = oracle.atmo(spec, lin, lt, lg, am[k], x, mode=1)
        f1 = oracle.atmo(spec, lin, lt, lg, am[k + 1], x, mode=1)
        assert oracle.atmo(spec, lin, lt, lg, m, x, mode=3) == pytest.approx(f0 + 0.41 * (f1 - f0), rel=1e-12)
        assert f0 == pytest.approx(cubic4_fn(lt, lg, am[k], x), rel=1e-11)
    for k in (3, 20, len(am) - 2):
        m = am[k] + 0.41 * (am[k + 1] - am[k])
        assert oracle.atmo(spec, lin, lt, lg, m, x, mode=3) == oracle.atmo(spec, lin, lt, lg, m, x, mode=1)


def steep_limb_fn(T, G, M, X):
    """Positive table with a steep rise off mu = 0 (nearly zero at the first
    two mu nodes, a plateau from the fourth): the cubic stencil over the
    first four nodes dips below zero between the second and third."""
    mu3 = AX[2][3]
    return (1.0 + 0.1 * (T - 6.0)) * (1e-6 + np.minimum(M / mu3, 1.0) ** 8) * (1.0 + 0.1 * X) + 0.0 * G


def test_strategy_b_clips_the_cubic_undershoot():
    """Strategy (b) equals max(0, (a)); on a steep limb the cubic of (a)
    undershoots below zero in the first mu intervals while the mixed (d)
    and (c) stay non-negative there (linear in the protected zone)."""
    spec, lin = make(steep_limb_fn)
    at, ag, am, ax = AX
    assert np.all(lin > 0)
    lt, lg, x = 6.0, 14.2, 0.5
    found = 0
    for k in range(4):
        for t in np.linspace(0.05, 0.95, 19):
            m = am[k] + t * (am[k + 1] - am[k])
            a = oracle.atmo(spec, lin, lt, lg, m, x, mode=1)
            b = oracle.atmo(spec, lin, lt, lg, m, x, mode=2)
            assert b == max(0.0, a)
            assert oracle.atmo(spec, lin, lt, lg, m, x, mode=0) >= 0.0
            assert oracle.atmo(spec, lin, lt, lg, m, x, mode=3) >= 0.0
            found += a < 0.0
    assert found > 0


@pytest.mark.parametrize("test", [1, 2])
def test_interpolation_tests_of_sect4_negative_samples(test):
    """The two small-hotspot geometries of the interpolation tests (Sect. 4,
    Table 3) on a synthetic steep-limb table: strategy (a) produces negative
    interpolated intensities where rays graze the limb, (b) counts the same
    ones and clips them, (c) and (d) produce none.  The flux bins stay
    positive here (the spot's cells span more than the steep mu range); with
    the paper's NSX-H table this diagnostic is parity unpinned."""
    spec, p = syn.interp_test_geometry(test)
    res = {}
    for mode in (0, 1, 2, 3):
        ft, _, d = oracle.forward(dict(spec, interp=mode), p)
        res[mode] = (d["n_negative"], ft)
    assert res[1][0] > 0 and res[2][0] == res[1][0]
    assert res[0][0] == 0 and res[3][0] == 0
    assert np.all(res[2][1] >= 0.0)
    # clipping only raises the flux relative to (a)
    assert np.all(res[2][1] >= res[1][1] - 1e-12 * np.abs(res[1][1]).max())
