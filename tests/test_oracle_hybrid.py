"""Pins of the oracle's close-pair hybrid step: the Kepler map of eq. (26) for
pairs whose step is not small against their own time scales, the eq. (28)
drift-kick-drift map for the rest (Sec. 1 names the idea, not a criterion).

The criterion against its definition in long double with square roots; the
limits (every pair close: the Kepler step; no pair close: leapfrog); a tight
binary solved exactly inside a hybrid step that kicks every other pair;
momentum; second order against RK4."""
import numpy as np
import pytest

from paper_1402_3325_amd import workloads
from tests import pins
from tests.test_oracle_step import _binary, _triple

LD = np.longdouble


def test_criterion_is_the_two_time_scale_test(oracle):
    """close <=> tau sqrt(mu/r^3) > eta or tau |W|/r > eta, evaluated in long
    double with square roots (cases within 1e-12 of the threshold skipped)."""
    rng = np.random.default_rng(21)
    checked = 0
    for _ in range(3000):
        X = rng.normal(size=3) * 10.0 ** rng.uniform(-4, 1)
        W = rng.normal(size=3) * 10.0 ** rng.uniform(-2, 1)
        mi, mj = 10.0 ** rng.uniform(-6, 0, 2)
        tau = 10.0 ** rng.uniform(-5, -1)
        eta = 10.0 ** rng.uniform(-3, 0)
        r = np.sqrt(np.sum(np.asarray(X, LD) ** 2))
        a = LD(tau) * np.sqrt(LD(mi + mj) / r ** 3) / LD(eta)
        b = LD(tau) * np.sqrt(np.sum(np.asarray(W, LD) ** 2)) / r / LD(eta)
        if abs(a - 1) < 1e-12 or abs(b - 1) < 1e-12:
            continue
        assert oracle.pair_is_close(tau, 1.0, mi, mj, X, W, eta) == bool(a > 1 or b > 1)
        checked += 1
    assert checked > 2900


def test_every_pair_close_is_the_kepler_step(oracle):
    m, r, v, tau = workloads.plummer(40, rng=np.random.default_rng(3))
    r1, v1, nk = oracle.step_hybrid(m, r, v, tau, 1e-30)
    r2, v2 = oracle.step(m, r, v, tau)
    assert nk == 40 * 39 // 2
    assert np.array_equal(r1, r2) and np.array_equal(v1, v2)


def test_no_pair_close_is_leapfrog(oracle):
    for seed in range(3):
        m, r, v, _ = workloads.plummer(32, rng=np.random.default_rng(seed))
        tau = 1e-3
        r1, v1, nk = oracle.step_hybrid(m, r, v, tau, 1e30)
        rl, vl = pins.leapfrog_dkd(m, r, v, tau)
        assert nk == 0
        assert np.max(np.abs(r1 - rl)) <= 4e-16 * np.abs(r).max()
        assert np.max(np.abs(v1 - vl)) <= 1e-14 * np.abs(v).max()


def test_rows_match_step(oracle):
    m, r, v, tau = workloads.cluster(n_stars=199, rng=np.random.default_rng(9))
    r1, v1, _ = oracle.step_hybrid(m, r, v, tau, 0.02)
    rows = np.array([0, 5, 77, 199])
    ro, vo = oracle.step_rows_hybrid(m, r, v, tau, 0.02, rows)
    assert np.array_equal(ro, r1[rows]) and np.array_equal(vo, v1[rows])


def _binary_and_star():
    """A binary (a = 1e-3, masses 0.5 and 0.3, e = 0.3) and a star of mass 0.2
    at distance 1 on a circular orbit about it."""
    rng = np.random.default_rng(31)
    mb, rb, vb = _binary(rng, 0.5, 0.3, 1e-3, 0.3)
    rb -= (mb[:, None] * rb).sum(0) / mb.sum()
    vb -= (mb[:, None] * vb).sum(0) / mb.sum()
    m = np.array([0.5, 0.3, 0.2])
    M = 1.0
    xo = np.array([1.0, 0.0, 0.0])
    wo = np.array([0.0, 1.0, 0.0]) * np.sqrt(M / 1.0)
    r = np.stack([rb[0] - 0.2 * xo, rb[1] - 0.2 * xo, 0.8 * xo])
    v = np.stack([vb[0] - 0.2 * wo, vb[1] - 0.2 * wo, 0.8 * wo])
    return m, r, v


def test_binary_is_solved_exactly_inside_the_hybrid(oracle):
    """With a step of a third of the binary's period, only the binary is a
    close pair; its relative orbit then follows the isolated Kepler orbit up to
    the tidal pull of the star (2.6e-7 of a over 10 steps here), as in the full
    Kepler step (2.4e-7), while leapfrog loses it (1.3 a)."""
    m, r, v = _binary_and_star()
    x0, w0 = r[0] - r[1], v[0] - v[1]
    P = 2 * np.pi * np.sqrt(1e-9 / 0.8)
    tau = P / 3
    rh, vh = r.copy(), v.copy()
    rk, vk = r.copy(), v.copy()
    for _ in range(10):
        rh, vh, nk = oracle.step_hybrid(m, rh, vh, tau, 0.05)
        assert nk == 1
        rk, vk = oracle.step(m, rk, vk, tau)
    rl, vl = r.copy(), v.copy()
    for _ in range(10):
        rl, vl = pins.leapfrog_dkd(m, rl, vl, tau)
    xe, _ = pins.kepler_elements(10 * tau, 0.8, x0, w0)
    xe = np.asarray(xe, dtype=np.float64)
    a = 1e-3
    err_h = np.linalg.norm((rh[0] - rh[1]) - xe) / a
    err_k = np.linalg.norm((rk[0] - rk[1]) - xe) / a
    err_l = np.linalg.norm((rl[0] - rl[1]) - xe) / a
    assert err_h < 1e-6 and err_k < 1e-6 and err_l > 0.1, (err_h, err_k, err_l)
    assert np.max(np.abs(rh - rk)) < 1e-9


def test_hybrid_conserves_momentum(oracle):
    m, r, v, tau = workloads.cluster(n_stars=63, rng=np.random.default_rng(4))
    P0 = (m[:, None] * v).sum(0)
    rr, vv = r, v
    for _ in range(5):
        rr, vv, _ = oracle.step_hybrid(m, rr, vv, tau, 0.01)
    pscale = (m * np.linalg.norm(v, axis=1)).sum()
    assert np.max(np.abs((m[:, None] * vv).sum(0) - P0)) <= 1e-14 * pscale


def test_hybrid_second_order(oracle):
    """Hierarchical triple at a fixed eta: the close pairs change with the step
    but each map is second order, so the global error falls as tau^2."""
    m, r, v = _triple()
    T = 0.25
    rr, _ = pins.rk4_nbody(m, r, v, T, 4000)
    errs = []
    for n in (320, 640, 1280):
        r1, v1 = r.copy(), v.copy()
        for _ in range(n):
            r1, v1, _ = oracle.step_hybrid(m, r1, v1, T / n, 0.01)
        errs.append(float(np.max(np.abs(r1 - np.asarray(rr, dtype=np.float64)))))
    assert 3.5 < errs[0] / errs[1] < 4.6 and 3.5 < errs[1] / errs[2] < 4.6, errs


def test_hybrid_rejects_bad_eta(oracle):
    m, r, v, tau = workloads.plummer(8, rng=np.random.default_rng(1))
    for eta in (0.0, -1.0, np.inf, np.nan):
        with pytest.raises(oracle.OracleError):
            oracle.step_hybrid(m, r, v, tau, eta)
