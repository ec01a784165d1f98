"""Pins of the oracle's learned-starter inputs and target (sref_guess_sample).

The learned starter is an extension of the method: the paper's solver only
needs a starting value for the universal variable.  The inputs are functions of
the three dimensionless numbers that fix a Kepler problem (tau', e', b') and the
target is y = log(chi r0 / (sqrt(mu) t)).  They are pinned here against
textbook orbital mechanics that the oracle does not use: the circular orbit,
Kepler's equation for elliptic and hyperbolic orbits in eccentric/hyperbolic
anomaly (solved by scipy's brentq), Barker's cubic for parabolas, the Kepler
scaling symmetry, time reversal, and the Taylor series of the root.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle

WIDE = [1e-9, 1e9, -1e9, 1e9]  # a domain that admits every test case


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q


def ellipse_state(mu, a, e, E0, rot):
    """State at eccentric anomaly E0 of the ellipse (a, e) around mass mu."""
    r0 = a * (1.0 - e * math.cos(E0))
    b = a * math.sqrt(1.0 - e * e)
    x = np.array([a * (math.cos(E0) - e), b * math.sin(E0), 0.0])
    k = math.sqrt(mu * a) / r0
    w = np.array([-k * math.sin(E0), k * math.sqrt(1.0 - e * e) * math.cos(E0), 0.0])
    return rot @ x, rot @ w


def hyperbola_state(mu, a, e, F0, rot):
    """State at hyperbolic anomaly F0 of the hyperbola (a < 0, e > 1)."""
    A = -a
    r0 = A * (e * math.cosh(F0) - 1.0)
    x = np.array([A * (e - math.cosh(F0)), A * math.sqrt(e * e - 1.0) * math.sinh(F0), 0.0])
    k = math.sqrt(mu * A) / r0
    w = np.array([-k * math.sinh(F0), k * math.sqrt(e * e - 1.0) * math.cosh(F0), 0.0])
    return rot @ x, rot @ w


def test_circular_orbit_target_is_zero():
    # r stays r0, so t = r0 s exactly and the root equals its free-drift value
    for taup in (0.01, 0.3, 1.0, 2.5, 3.1):
        mu, r = 2.7, 0.8
        x0 = [r, 0.0, 0.0]
        w0 = [0.0, math.sqrt(mu / r), 0.0]
        t = taup / math.sqrt(mu / r**3)
        feat, y, ind = oracle.guess_sample(t, mu, x0, w0, WIDE)
        assert ind
        assert abs(y) < 1e-14
        assert abs(feat[1]) < 1e-15 and abs(feat[2] - 1.0) < 1e-15
        assert feat[3] == pytest.approx(taup, rel=1e-14)
        assert feat[6] == pytest.approx(taup, rel=1e-14)  # mean anomaly advance, b' = 1
        assert abs(feat[7]) < 1e-15


@pytest.mark.parametrize("e", [0.05, 0.4, 0.9, 0.99])
def test_elliptic_against_keplers_equation(e):
    rng = np.random.default_rng(int(e * 1000))
    for _ in range(20):
        mu = 10 ** rng.uniform(-4, 1)
        a = 10 ** rng.uniform(-3, 2)
        E0 = rng.uniform(-math.pi, math.pi)
        x0, w0 = ellipse_state(mu, a, e, E0, _rot(rng))
        n = math.sqrt(mu / a**3)
        M = rng.uniform(-0.98, 0.98) * math.pi  # mean anomaly advance within half a period
        t = M / n
        # Kepler's equation for the change dE of eccentric anomaly
        g = lambda d: d - e * math.cos(E0) * math.sin(d) + e * math.sin(E0) * (1 - math.cos(d)) - M
        dE = brentq(g, -2 * math.pi, 2 * math.pi, xtol=1e-300, rtol=9e-16, maxiter=500)
        chi = math.sqrt(a) * dE  # universal variable of an ellipse
        r0 = a * (1 - e * math.cos(E0))
        y_ref = math.log(chi * r0 / (math.sqrt(mu) * t))
        feat, y, ind = oracle.guess_sample(t, mu, x0, w0, WIDE)
        assert ind
        # conditioning: dE is fixed to ~1e-16 relative, y inherits it
        assert abs(y - y_ref) <= 2e-12 * (1 + abs(y_ref)), (e, E0, M, y, y_ref)
        sg = math.copysign(1.0, t)
        assert 1.0 - feat[2] == pytest.approx(e * math.cos(E0), abs=1e-12)  # e cos E0
        assert feat[7] == pytest.approx(sg * e * math.sin(E0), abs=1e-12)  # e sin E0
        # mean anomaly advance; b' = r0 / a is recovered from 2 - r0 |w0|^2 / mu, which
        # cancels near pericenter of eccentric orbits (the state itself carries ~eps)
        assert feat[6] == pytest.approx(abs(M), rel=1e-13 * a / r0)
        assert feat[1] == pytest.approx(sg * e * math.sin(E0) * math.sqrt(a / r0), abs=1e-12)
        assert feat[3] == pytest.approx(abs(t) * math.sqrt(mu / r0**3), rel=1e-13)


@pytest.mark.parametrize("e", [1.01, 1.5, 4.0])
def test_hyperbolic_against_keplers_equation(e):
    rng = np.random.default_rng(int(e * 100))
    for _ in range(20):
        mu = 10 ** rng.uniform(-4, 1)
        a = -(10 ** rng.uniform(-3, 1))
        F0 = rng.uniform(-3, 3)
        x0, w0 = hyperbola_state(mu, a, e, F0, _rot(rng))
        n = math.sqrt(mu / (-a) ** 3)
        t = rng.uniform(-3, 3) / n
        Mh = n * t
        g = lambda d: e * math.sinh(F0 + d) - e * math.sinh(F0) - d - Mh
        lo, hi = (0.0, 1.0) if Mh > 0 else (-1.0, 0.0)
        while g(hi) < 0:
            hi *= 2
        while g(lo) > 0:
            lo *= 2
        dF = brentq(g, lo, hi, xtol=1e-300, rtol=9e-16, maxiter=500)
        chi = math.sqrt(-a) * dF  # universal variable of a hyperbola
        r0 = -a * (e * math.cosh(F0) - 1)
        y_ref = math.log(chi * r0 / (math.sqrt(mu) * t))
        feat, y, ind = oracle.guess_sample(t, mu, x0, w0, WIDE)
        assert ind
        assert abs(y - y_ref) <= 2e-12 * (1 + abs(y_ref)), (e, F0, t, y, y_ref)
        assert 1.0 - feat[2] == pytest.approx(e * math.cosh(F0), rel=1e-12)
        assert feat[6] == 0.0 and feat[7] == 0.0


def test_parabolic_against_barkers_cubic():
    rng = np.random.default_rng(7)
    for _ in range(30):
        mu = 10 ** rng.uniform(-3, 1)
        r0 = 10 ** rng.uniform(-2, 1)
        v = math.sqrt(2 * mu / r0)  # escape speed: alpha = 0
        ang = rng.uniform(0.05, math.pi - 0.05)  # angle between x0 and w0
        rot = _rot(rng)
        x0 = rot @ np.array([r0, 0.0, 0.0])
        w0 = rot @ np.array([v * math.cos(ang), v * math.sin(ang), 0.0])
        t = rng.uniform(-5, 5) * math.sqrt(r0**3 / mu)
        # sqrt(mu) t = r0 chi + sigma0 chi^2 / 2 + chi^3 / 6 with sigma0 = x0.w0 / sqrt(mu)
        sig0 = float(x0 @ w0) / math.sqrt(mu)
        roots = np.roots([1 / 6, sig0 / 2, r0, -math.sqrt(mu) * t])
        real = roots[np.abs(roots.imag) < 1e-9 * np.abs(roots).max()].real
        chi = real[np.argmin(np.abs(real - math.sqrt(mu) * t / r0))] if len(real) > 1 else real[0]
        chi = brentq(lambda c: c**3 / 6 + sig0 * c * c / 2 + r0 * c - math.sqrt(mu) * t,
                     chi - 1e-6 * (1 + abs(chi)), chi + 1e-6 * (1 + abs(chi)), rtol=9e-16)
        y_ref = math.log(chi * r0 / (math.sqrt(mu) * t))
        feat, y, ind = oracle.guess_sample(t, mu, x0, w0, WIDE)
        assert ind
        assert abs(feat[2]) < 1e-13  # b' = 0 up to the rounding of |w0|^2
        assert abs(y - y_ref) <= 1e-10 * (1 + abs(y_ref)), (t, y, y_ref)


def test_taylor_series_of_the_root():
    # chi' = tau' - e' tau'^2 / 2 + (3 e'^2 - 1 + b') tau'^3 / 6 + O(tau'^4), so
    # exp(y) - 1 + feat[4] / 2 - feat[5] = O(tau'^3): a wrong sign or a dropped
    # term in feat[4] or feat[5] leaves an O(tau') or O(tau'^2) residual.
    rng = np.random.default_rng(11)
    for _ in range(50):
        mu = 10 ** rng.uniform(-3, 1)
        x0 = rng.normal(size=3)
        w0 = rng.normal(size=3) * math.sqrt(mu / np.linalg.norm(x0)) * rng.uniform(0.2, 1.6)
        r0 = np.linalg.norm(x0)
        for taup in (1e-3, 2e-3):
            t = taup * math.sqrt(r0**3 / mu) * rng.choice([-1, 1])
            feat, y, ind = oracle.guess_sample(t, mu, x0, w0, WIDE)
            assert ind
            res = math.expm1(y) + feat[4] / 2 - feat[5]
            scale = 1 + abs(feat[1]) ** 3 + abs(feat[2]) ** 2
            assert abs(res) <= 2 * scale * taup**3, (taup, res)


def test_kepler_scaling_invariance():
    # x -> lam x, mu -> kap mu, w -> sqrt(kap/lam) w, t -> lam^(3/2) / sqrt(kap) t maps
    # Kepler orbits onto Kepler orbits: inputs and target are unchanged.
    rng = np.random.default_rng(3)
    for _ in range(40):
        mu = 10 ** rng.uniform(-3, 1)
        x0 = rng.normal(size=3)
        w0 = rng.normal(size=3) * math.sqrt(mu / np.linalg.norm(x0)) * rng.uniform(0.2, 1.8)
        t = rng.uniform(-4, 4) * math.sqrt(np.linalg.norm(x0) ** 3 / mu)
        lam, kap = 10 ** rng.uniform(-3, 3), 10 ** rng.uniform(-3, 3)
        f1, y1, i1 = oracle.guess_sample(t, mu, x0, w0, WIDE)
        f2, y2, i2 = oracle.guess_sample(t * lam**1.5 / math.sqrt(kap), mu * kap, lam * x0,
                                         math.sqrt(kap / lam) * w0, WIDE)
        assert i1 and i2
        np.testing.assert_allclose(f2, f1, rtol=1e-12, atol=1e-12)
        assert abs(y2 - y1) <= 1e-11 * (1 + abs(y1))


def test_time_reversal():
    # The flow backwards from (x0, w0) is the flow forwards from (x0, -w0) with the
    # velocity flipped, so chi(-t; w0) = -chi(t; -w0): inputs and target agree.
    rng = np.random.default_rng(5)
    for _ in range(40):
        mu = 10 ** rng.uniform(-3, 1)
        x0 = rng.normal(size=3)
        w0 = rng.normal(size=3) * math.sqrt(mu / np.linalg.norm(x0)) * rng.uniform(0.2, 1.8)
        t = rng.uniform(0.01, 4) * math.sqrt(np.linalg.norm(x0) ** 3 / mu)
        f1, y1, i1 = oracle.guess_sample(-t, mu, x0, w0, WIDE)
        f2, y2, i2 = oracle.guess_sample(t, mu, x0, -w0, WIDE)
        assert i1 and i2
        np.testing.assert_allclose(f1, f2, rtol=1e-14, atol=0)
        assert abs(y1 - y2) <= 1e-13 * (1 + abs(y1))


def test_period_reduction_and_domain():
    mu, a, e = 1.0, 1.0, 0.6
    rng = np.random.default_rng(9)
    x0, w0 = ellipse_state(mu, a, e, 0.7, _rot(rng))
    P = 2 * math.pi * math.sqrt(a**3 / mu)
    f1, y1, _ = oracle.guess_sample(0.9, mu, x0, w0, WIDE)
    f2, y2, _ = oracle.guess_sample(0.9 + 3 * P, mu, x0, w0, WIDE)
    np.testing.assert_allclose(f2, f1, rtol=1e-12, atol=1e-12)
    assert abs(y2 - y1) < 1e-12
    # the domain bounds are inclusive and every bound excludes
    taup = f1[3]
    assert oracle.guess_sample(0.9, mu, x0, w0, [taup, taup, -1e9, 1e9])[2]
    assert not oracle.guess_sample(0.9, mu, x0, w0, [taup * 1.001, 1e9, -1e9, 1e9])[2]
    assert not oracle.guess_sample(0.9, mu, x0, w0, [1e-9, taup * 0.999, -1e9, 1e9])[2]
    assert not oracle.guess_sample(0.9, mu, x0, w0, [1e-9, 1e9, f1[2] * 1.001, 1e9])[2]
    assert not oracle.guess_sample(0.9, mu, x0, w0, [1e-9, 1e9, -1e9, abs(f1[1]) * 0.999])[2]
    # no Kepler problem without mass, and none at t = 0
    assert not oracle.guess_sample(0.9, 0.0, x0, w0, WIDE)[2]
    assert not oracle.guess_sample(0.0, mu, x0, w0, WIDE)[2]
