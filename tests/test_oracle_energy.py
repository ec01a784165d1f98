"""Pins of the oracle's diagnostics (eqs. 1-3: kinetic and potential energy,
plus linear and angular momentum and the centre of mass) and of the weights of
the triple jump (the higher-order composition Sec. 2.2 proposes).

Every expected value here comes from a closed form written out in the test:
the two-body energy -G m1 m2 / (2a) and angular momentum mu_red sqrt(G M a
(1 - e^2)) along the orbit normal, the potential of regular polygons and
polyhedra by hand, the change of P, L and R_cm under a Galilean boost and a
translation, and the virial scaling of the input generator's Plummer sphere
(its own direct sum, independent of the oracle).  The triple jump is checked
bitwise against three merged steps at weights computed in 50-digit decimal
arithmetic.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from paper_1402_3325_amd import workloads

E, K, U = 0, 1, 2
P = slice(3, 6)
L = slice(6, 9)
RCM = slice(9, 12)


def _energy(oracle, m, r, v, G=1.0):
    """The oracle's diagnostics as one array {E, K, U, P[3], L[3], R_cm[3]}."""
    d = oracle.energy(m, r, v, G)
    return np.concatenate([[d["E"], d["K"], d["U"]], d["P"], d["L"], d["Rcm"]])


def _two_body(m1, m2, a, e, inc, Om, om, M, G=1.0):
    """Barycentric state of a bound pair from its relative orbit's elements."""
    mu = G * (m1 + m2)
    X, W = workloads.elements_to_state(mu, a, e, inc, Om, om, M)
    m = np.array([m1, m2])
    f1, f2 = m2 / (m1 + m2), m1 / (m1 + m2)
    r = np.stack([f1 * X, -f2 * X])
    v = np.stack([f1 * W, -f2 * W])
    return m, r, v


@pytest.mark.parametrize("m1,m2,a,e,G", [(1.0, 1e-3, 1.0, 0.0, 1.0), (0.7, 0.3, 0.01, 0.9, 1.0),
                                         (2.0, 5.0, 3.5, 0.4, 0.25), (1e-5, 1e-5, 1e-4, 0.99, 1.0)])
def test_two_body_energy_and_angular_momentum(oracle, m1, m2, a, e, G):
    """E = -G m1 m2 / (2a) at every phase; L = mu_red sqrt(G M a (1 - e^2)) n,
    n = (sin i sin Om, -sin i cos Om, cos i) the orbit normal; P = 0 and
    R_cm = 0 in the barycentric frame; K = mu_red |W|^2 / 2, U = -G m1 m2 / r."""
    inc, Om, om = 0.3, 1.1, 2.0
    mred = m1 * m2 / (m1 + m2)
    for M in (0.0, 1.0, 2.5, 4.0):
        m, r, v = _two_body(m1, m2, a, e, inc, Om, om, M, G)
        out = _energy(oracle, m, r, v, G)
        X, W = r[0] - r[1], v[0] - v[1]
        rr = math.sqrt(float(X @ X))
        scale = G * m1 * m2 / rr
        assert abs(out[E] - (-G * m1 * m2 / (2 * a))) <= 1e-14 * scale
        assert abs(out[K] - 0.5 * mred * float(W @ W)) <= 1e-14 * abs(out[K]) + 1e-300
        assert abs(out[U] - (-G * m1 * m2 / rr)) <= 1e-14 * scale
        Lmag = mred * math.sqrt(G * (m1 + m2) * a * (1 - e * e))
        n = np.array([math.sin(inc) * math.sin(Om), -math.sin(inc) * math.cos(Om), math.cos(inc)])
        assert np.max(np.abs(out[L] - Lmag * n)) <= 1e-13 * Lmag
        pscale = mred * math.sqrt(float(W @ W))
        assert np.max(np.abs(out[P])) <= 1e-15 * pscale
        assert np.max(np.abs(out[RCM])) <= 1e-15 * rr


def test_circular_orbit_angular_momentum_sign(oracle):
    """A prograde circular orbit in the xy plane: L_z = +mu_red sqrt(G M a),
    L_x = L_y = 0; reversing the velocities flips the sign of L_z alone."""
    m1, m2, a, G = 1.0, 0.25, 2.0, 1.0
    mu = G * (m1 + m2)
    vc = math.sqrt(mu / a)
    m = np.array([m1, m2])
    f1, f2 = m2 / (m1 + m2), m1 / (m1 + m2)
    r = np.array([[f1 * a, 0.0, 0.0], [-f2 * a, 0.0, 0.0]])
    v = np.array([[0.0, f1 * vc, 0.0], [0.0, -f2 * vc, 0.0]])
    Lz = m1 * m2 / (m1 + m2) * math.sqrt(mu * a)
    out = _energy(oracle, m, r, v, G)
    assert abs(out[8] - Lz) <= 1e-15 * Lz and out[6] == 0.0 and out[7] == 0.0
    assert abs(out[E] - (-G * m1 * m2 / (2 * a))) <= 1e-15 * G * m1 * m2 / a
    out2 = _energy(oracle, m, r, -v, G)
    assert abs(out2[8] + Lz) <= 1e-15 * Lz


def test_potential_of_regular_figures_by_hand(oracle):
    """U of an equilateral triangle (side s, unequal masses), a square of
    equal masses and a regular tetrahedron, each written out pair by pair;
    K, P, L vanish at rest, R_cm is the mass-weighted centre."""
    s = 0.37
    m = np.array([0.2, 0.5, 1.3])
    r = np.array([[0.0, 0.0, 0.0], [s, 0.0, 0.0], [0.5 * s, 0.5 * math.sqrt(3.0) * s, 0.0]])
    v = np.zeros_like(r)
    G = 2.0
    out = _energy(oracle, m, r, v, G)
    U3 = -G * (0.2 * 0.5 + 0.2 * 1.3 + 0.5 * 1.3) / s
    assert abs(out[U] - U3) <= 1e-15 * abs(U3)
    assert out[K] == 0.0 and np.all(out[P] == 0.0) and np.all(out[L] == 0.0)
    assert abs(out[E] - U3) <= 1e-15 * abs(U3)
    rc = (m[:, None] * r).sum(0) / m.sum()
    assert np.max(np.abs(out[RCM] - rc)) <= 1e-16

    m4 = np.full(4, 0.25)
    r4 = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    # four sides of length sqrt(2) and two diagonals of length 2
    U4 = -(0.25 * 0.25) * (4.0 / math.sqrt(2.0) + 2.0 / 2.0)
    assert abs(_energy(oracle, m4, r4, np.zeros_like(r4))[U] - U4) <= 1e-15 * abs(U4)

    rt = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
    mt = np.array([1.0, 2.0, 3.0, 4.0])
    # all six edges have length 2 sqrt(2)
    pairs = sum(mt[i] * mt[j] for i in range(4) for j in range(i + 1, 4))
    Ut = -pairs / (2.0 * math.sqrt(2.0))
    assert abs(_energy(oracle, mt, rt, np.zeros_like(rt))[U] - Ut) <= 1e-15 * abs(Ut)


def test_boost_and_translation(oracle):
    """Shifting every position by D and every velocity by V (from a
    barycentric state with P = 0): P = M V, R_cm = D, K grows by M |V|^2 / 2,
    U is unchanged, and L grows by M D x V."""
    rng = np.random.default_rng(7)
    m, r, v, _ = workloads.plummer(64, rng=rng)
    r, v = r - (m[:, None] * r).sum(0) / m.sum(), v - (m[:, None] * v).sum(0) / m.sum()
    base = _energy(oracle, m, r, v)
    D = np.array([0.3, -1.2, 0.7])
    V = np.array([-0.05, 0.02, 0.11])
    out = _energy(oracle, m, r + D, v + V)
    M = m.sum()
    assert np.max(np.abs(out[P] - M * V)) <= 1e-15
    assert np.max(np.abs(out[RCM] - D)) <= 1e-15
    assert abs(out[U] - base[U]) <= 1e-14 * abs(base[U])
    assert abs(out[K] - (base[K] + 0.5 * M * float(V @ V))) <= 1e-14 * out[K]
    assert np.max(np.abs(out[L] - (base[L] + M * np.cross(D, V)))) <= 1e-14


def test_plummer_sphere_virial_scaling(oracle):
    """The input generator rescales its Plummer sphere with its own direct sum
    to 2K = |U| and E = -1/4 (Henon units); the oracle's diagnostics agree."""
    m, r, v, _ = workloads.plummer(512, rng=np.random.default_rng(9))
    out = _energy(oracle, m, r, v)
    assert abs(out[E] + 0.25) <= 1e-13
    assert abs(2.0 * out[K] + out[U]) <= 1e-13
    assert abs(out[U] + 0.5) <= 1e-13


def test_energy_g_scales_potential_only(oracle):
    m, r, v, _ = workloads.plummer(40, rng=np.random.default_rng(4))
    a = _energy(oracle, m, r, v, 1.0)
    b = _energy(oracle, m, r, v, 3.0)
    assert b[K] == a[K] and np.array_equal(b[3:], a[3:])
    assert abs(b[U] - 3.0 * a[U]) <= 1e-15 * abs(b[U])


def _yoshida_weights():
    """g1 = 1/(2 - 2^(1/3)) and g0 = 1 - 2 g1 (Yoshida 1990), in 50 digits;
    g1 as its correctly rounded double."""
    getcontext().prec = 50
    c = Decimal(2) ** (Decimal(1) / Decimal(3))
    g1 = Decimal(1) / (Decimal(2) - c)
    return g1, Decimal(1) - 2 * g1


def test_yoshida_weights_conditions():
    g1, g0 = _yoshida_weights()
    assert abs(2 * g1 + g0 - 1) < Decimal(10) ** -45
    assert abs(2 * g1 ** 3 + g0 ** 3) < Decimal(10) ** -45
    # the double weights: g0 = 1 - 2 g1 is exact in double arithmetic
    d1 = float(g1)
    assert Decimal(1.0 - 2.0 * d1) == Decimal(1) - 2 * Decimal(d1)


def test_triple_jump_is_three_merged_steps_at_yoshida_weights(oracle):
    """One triple-jump step over tau equals, bitwise, the merged steps over
    g1 tau, g0 tau, g1 tau with the weights of the 50-digit evaluation."""
    g1, _ = _yoshida_weights()
    d1 = float(g1)
    d0 = 1.0 - 2.0 * d1
    for m, r, v, tau in (workloads.planetary(rng=np.random.default_rng(3)),
                         workloads.plummer(48, rng=np.random.default_rng(5))):
        r1, v1 = r.copy(), v.copy()
        r1, v1 = oracle.evolve_scheme(m, r1, v1, tau, 2, oracle.SCHEME_TRIPLE_JUMP)
        r2, v2 = r.copy(), v.copy()
        for _ in range(2):
            for w in (d1, d0, d1):
                r2, v2 = oracle.step(m, r2, v2, w * tau)
        assert np.array_equal(r1, r2) and np.array_equal(v1, v2)
