"""Pins of the inequalities the stack's checkpoint prediction relies on,
checked on the oracle's exact two-body states (no GPU).

For an elliptic orbit with perihelion distance q = a (1 - e) and perihelion
speed vmax = n a sqrt((1 + e) / (1 - e)), the third derivative of the
heliocentric position obeys |r'''| <= 2 mu vmax / q^3, so the second-order
prediction r + v D + (a/2) D^2 from the state at t is within
(2 mu vmax / q^3) D^3 / 6 of r(t + D); and the light time changes by at most
(vmax + vobs) D / (c - vmax) over D days for an observer slower than vobs."""
import math

import numpy as np
import pytest

import oracle

MU = 0.01720209895 ** 2
C_AU_DAY = 299792458.0 * 86400.0 / 149597870700.0


def _orbits(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.6, 4.0, n), rng.uniform(0.0, 0.95, n), rng.uniform(0.0, math.pi, n),
                     rng.uniform(0.0, 2 * math.pi, n), rng.uniform(0.0, 2 * math.pi, n),
                     rng.uniform(0.0, 2 * math.pi, n)], 1)


def _vmax_q(el):
    a, e = el[0], el[1]
    n = 0.01720209895 / a ** 1.5
    return n * a * math.sqrt((1 + e) / (1 - e)), a * (1 - e)


def test_second_order_prediction_within_the_jerk_bound(oracle_lib):
    rng = np.random.default_rng(11)
    worst = 0.0
    for el in _orbits(200, 3):
        vmax, q = _vmax_q(el)
        J = 2.0 * MU * vmax / q ** 3
        for _ in range(5):
            t = rng.uniform(-100.0, 100.0)
            D = rng.uniform(0.0, 30.0)
            r0, v0, _ = oracle.helio_state(el, 0.0, t)
            r1, _, _ = oracle.helio_state(el, 0.0, t + D)
            acc = -MU * r0 / np.linalg.norm(r0) ** 3
            err = np.linalg.norm(r1 - (r0 + v0 * D + 0.5 * acc * D * D))
            bound = J * D ** 3 / 6.0
            assert err <= bound * (1 + 1e-9) + 1e-13, (el, t, D, err, bound)
            worst = max(worst, err / max(bound, 1e-300))
    # the bound is not vacuous: some cases come within a factor of a few of it
    assert worst > 0.05


def test_speed_and_jerk_bounds_hold_along_the_orbit(oracle_lib):
    # |v| <= vmax everywhere; |d/dt (r / |r|^3)| <= 2 |v| / r^3 (by central differences of the exact state)
    for el in _orbits(100, 5):
        vmax, q = _vmax_q(el)
        for t in np.linspace(-200.0, 200.0, 9):
            r, v, _ = oracle.helio_state(el, 0.0, t)
            assert np.linalg.norm(v) <= vmax * (1 + 1e-12)
            assert np.linalg.norm(r) >= q * (1 - 1e-12)
            h = 1e-3
            f = lambda s: oracle.helio_state(el, 0.0, s)[0] / np.linalg.norm(oracle.helio_state(el, 0.0, s)[0]) ** 3
            d = (f(t + h) - f(t - h)) / (2 * h)
            rn = np.linalg.norm(r)
            assert np.linalg.norm(d) <= 2.0 * np.linalg.norm(v) / rn ** 3 * (1 + 1e-5)


@pytest.mark.parametrize("seed", [1, 2])
def test_light_time_change_bound(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    w_obs = 2 * math.pi / 365.25  # an observer on a 1 AU circle: speed 0.0172 AU/day
    vobs = w_obs * 1.0
    obs = lambda t: np.array([math.cos(w_obs * t), math.sin(w_obs * t), 0.0])
    for el in _orbits(60, seed):
        vmax, _ = _vmax_q(el)
        for _ in range(4):
            t = rng.uniform(-50.0, 50.0)
            D = rng.uniform(0.0, 30.0)
            _, tau0, _, st0 = oracle.light_time(el, 0.0, t, obs(t))
            _, tau1, _, st1 = oracle.light_time(el, 0.0, t + D, obs(t + D))
            assert abs(tau1 - tau0) <= (vmax + vobs) * D / (C_AU_DAY - vmax) * (1 + 1e-9) + 1e-15
