"""Seeded synthetic initial conditions for the Sakura step.

This module holds only input generation (sampling, orbital elements to
Cartesian, unit rescaling); none of the integrator's arithmetic.  Both the HIP
path's tests/benchmark and the CPU oracle's tests draw their inputs from here,
so the two sides always see identical bytes.

Workloads (G = 1 throughout):

* ``planetary``  -- a star of mass 1 with planets on near-circular, near-coplanar
  orbits (masses log-uniform in [1e-5, 1e-3], a log-uniform in [1, 30],
  e ~ U[0, 0.1], i ~ U[0, 0.05]); tau = innermost period / 64.  Stands in for the
  Sun-with-planets test of Sec. 3.1, whose initial conditions are not used here.
* ``plummer``    -- equal-mass Plummer sphere in Henon units (E = -1/4), sampled
  with the Aarseth, Henon & Wielen (1974) recipe; the workload of the scaling
  tests of Sec. 4.
* ``cluster``    -- 16383 stars of total mass 1 (10 % of them in primordial
  binaries with a log-uniform in [1e-4, 1e-2] and thermal eccentricities) around
  a central point mass 0.01: a star cluster with a central black hole and
  primordial binaries, the regimes the abstract and Sec. 3.2 single out.
* ``ensemble``   -- many independent planetary systems of uneven size in CSR
  layout.
* ``plummer_bh`` -- a 128-star Plummer sphere around a black hole of q star
  masses, q = 1 .. 1e12: the mass-ratio accuracy study of Sec. 3.2.
* ``hierarchical4`` -- two circular binaries on a circular outer orbit,
  a_out/a_in = 10 .. 1000: the hierarchical accuracy test of Sec. 3.1.
* ``test_particles`` -- one massive body plus massless particles (each follows an
  exact two-body orbit under the method).
* ``kepler_cases``   -- random two-body states (elliptic, hyperbolic,
  near-parabolic, highly eccentric) for checks of the pair solver.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 14023325


def rng_for(config: int, offset: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config + offset))


# --------------------------------------------------------------------------
# Orbital elements -> Cartesian (initial-condition construction only)
# --------------------------------------------------------------------------
def _eccentric_anomaly(M, e):
    """Solve M = E - e sin E for bound orbits (vectorised Newton)."""
    M = np.mod(M, 2.0 * np.pi)
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(60):
        d = (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        E = E - d
        if np.all(np.abs(d) < 1e-15):
            break
    return E


def _rotation(inc, Om, om):
    """Matrices Rz(Om) Rx(inc) Rz(om), shape [..., 3, 3]."""
    cO, sO = np.cos(Om), np.sin(Om)
    ci, si = np.cos(inc), np.sin(inc)
    co, so = np.cos(om), np.sin(om)
    R = np.empty(np.shape(inc) + (3, 3))
    R[..., 0, 0] = cO * co - sO * so * ci
    R[..., 0, 1] = -cO * so - sO * co * ci
    R[..., 0, 2] = sO * si
    R[..., 1, 0] = sO * co + cO * so * ci
    R[..., 1, 1] = -sO * so + cO * co * ci
    R[..., 1, 2] = -cO * si
    R[..., 2, 0] = so * si
    R[..., 2, 1] = co * si
    R[..., 2, 2] = ci
    return R


def elements_to_state(mu, a, e, inc, Om, om, M):
    """Relative position and velocity of bound orbits from classical elements."""
    mu, a, e, inc, Om, om, M = np.broadcast_arrays(
        *[np.asarray(x, dtype=np.float64) for x in (mu, a, e, inc, Om, om, M)])
    E = _eccentric_anomaly(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    n = np.sqrt(mu / a ** 3)
    den = 1.0 - e * cE
    p = np.stack([a * (cE - e), a * b * sE, np.zeros_like(a)], axis=-1)
    q = np.stack([-a * n * sE / den, a * n * b * cE / den, np.zeros_like(a)], axis=-1)
    R = _rotation(inc, Om, om)
    return np.einsum("...ij,...j->...i", R, p), np.einsum("...ij,...j->...i", R, q)


def _isotropic(rng, n):
    c = rng.uniform(-1.0, 1.0, n)
    s = np.sqrt(1.0 - c * c)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.stack([s * np.cos(ph), s * np.sin(ph), c], axis=-1)


def _to_com_frame(m, r, v):
    M = m.sum()
    r = r - (m[:, None] * r).sum(0) / M
    v = v - (m[:, None] * v).sum(0) / M
    return r, v


def potential_energy(m, r, G=1.0, chunk=1024):
    """Direct-sum potential energy (used only to rescale initial conditions)."""
    n = m.shape[0]
    U = 0.0
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d = r[s:e, None, :] - r[None, :, :]
        d2 = np.einsum("ijk,ijk->ij", d, d)
        idx = np.arange(s, e)
        d2[idx - s, idx] = np.inf
        U -= 0.5 * np.sum(m[s:e, None] * m[None, :] / np.sqrt(d2))
    return G * U


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def planetary(n_planets=15, rng=None, seed=None):
    """Star (mass 1) + planets; returns m, r, v, tau (barycentric frame)."""
    if rng is None:
        rng = rng_for(0) if seed is None else np.random.Generator(np.random.PCG64(seed))
    k = n_planets
    mp = 10.0 ** rng.uniform(-5.0, -3.0, k)
    a = 10.0 ** rng.uniform(0.0, np.log10(30.0), k)
    e = rng.uniform(0.0, 0.1, k)
    inc = rng.uniform(0.0, 0.05, k)
    Om, om, M = (rng.uniform(0.0, 2.0 * np.pi, k) for _ in range(3))
    x, w = elements_to_state(1.0 + mp, a, e, inc, Om, om, M)
    m = np.concatenate([[1.0], mp])
    r = np.concatenate([np.zeros((1, 3)), x])
    v = np.concatenate([np.zeros((1, 3)), w])
    r, v = _to_com_frame(m, r, v)
    i = np.argmin(a)
    tau = 2.0 * np.pi * np.sqrt(a[i] ** 3 / (1.0 + mp[i])) / 64.0
    return m, r, v, float(tau)


def _plummer_raw(n, rng, mass_cut=0.999):
    """Plummer sphere (G = M = 1, scale 1) by Aarseth, Henon & Wielen (1974)."""
    X1 = rng.uniform(0.0, mass_cut, n)
    X1 = np.maximum(X1, 1e-12)
    rad = 1.0 / np.sqrt(X1 ** (-2.0 / 3.0) - 1.0)
    r = rad[:, None] * _isotropic(rng, n)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        X4 = rng.uniform(0.0, 1.0, todo.size)
        X5 = rng.uniform(0.0, 1.0, todo.size)
        ok = 0.1 * X5 < X4 * X4 * (1.0 - X4 * X4) ** 3.5
        q[todo[ok]] = X4[ok]
        todo = todo[~ok]
    ve = np.sqrt(2.0) * (1.0 + rad * rad) ** (-0.25)
    v = (q * ve)[:, None] * _isotropic(rng, n)
    return r, v


def _virialise_henon(m, r, v, G=1.0):
    """Rescale to 2K = |U| and E = -1/4 (Henon units)."""
    r, v = _to_com_frame(m, r, v)
    U = potential_energy(m, r, G)
    r = r * (U / -0.5)
    K = 0.5 * np.sum(m * np.einsum("ij,ij->i", v, v))
    v = v * np.sqrt(0.25 / K)
    return r, v


def plummer(n=4096, rng=None):
    """Equal-mass Plummer sphere in Henon units; returns m, r, v, tau."""
    if rng is None:
        rng = rng_for(1)
    r, v = _plummer_raw(n, rng)
    r *= 3.0 * np.pi / 16.0
    v *= np.sqrt(16.0 / (3.0 * np.pi))
    m = np.full(n, 1.0 / n)
    r, v = _virialise_henon(m, r, v)
    return m, r, v, 1.0 / 1024.0


def cluster(n_stars=16383, binary_fraction=0.1, m_bh=0.01, rng=None):
    """Plummer cluster with primordial binaries around a central point mass.

    Returns m, r, v, tau with the central mass at index 0."""
    if rng is None:
        rng = rng_for(2)
    n_bin = int(round(binary_fraction * n_stars / 2.0))
    n_cen = n_stars - n_bin
    ms = 1.0 / n_stars
    mc = np.full(n_cen, ms)
    which = rng.permutation(n_cen)[:n_bin]
    mc[which] = 2.0 * ms
    rc, vc = _plummer_raw(n_cen, rng)
    rc *= 3.0 * np.pi / 16.0
    vc *= np.sqrt(16.0 / (3.0 * np.pi))
    rc, vc = _virialise_henon(mc / mc.sum(), rc, vc)
    # Binaries: relative orbits about each chosen centre of mass.
    a = 10.0 ** rng.uniform(-4.0, -2.0, n_bin)
    e = np.sqrt(rng.uniform(0.0, 1.0, n_bin))
    inc = np.arccos(rng.uniform(-1.0, 1.0, n_bin))
    Om, om, M = (rng.uniform(0.0, 2.0 * np.pi, n_bin) for _ in range(3))
    x, w = elements_to_state(2.0 * ms, a, e, inc, Om, om, M)
    single = np.setdiff1d(np.arange(n_cen), which)
    m = np.concatenate([[m_bh], np.full(single.size, ms), np.full(2 * n_bin, ms)])
    r = np.concatenate([np.zeros((1, 3)), rc[single],
                        rc[which] + 0.5 * x, rc[which] - 0.5 * x])
    v = np.concatenate([np.zeros((1, 3)), vc[single],
                        vc[which] + 0.5 * w, vc[which] - 0.5 * w])
    # Interleave binary members so each binary sits in one tile of the pair loop
    # as often as the single stars do: shuffle all stars, keep the central mass
    # first.
    perm = np.concatenate([[0], 1 + rng.permutation(n_stars)])
    m, r, v = m[perm], r[perm], v[perm]
    r, v = _to_com_frame(m, r, v)
    return m, r, v, 1.0 / 2048.0


def plummer_bh(n_stars=128, q=1.0e6, rng=None):
    """Plummer sphere of n_stars equal-mass stars around a central black hole
    of q star masses (the mass-ratio study of Sec. 3.2): G = 1, total mass 1,
    the stars at the Henon length scale of a Plummer sphere, centre of mass at
    rest, and the velocities scaled to virial equilibrium, 2K = |U| (so E =
    U/2; the length scale is not stretched to E = -1/4, which for large q
    would shrink the system until the stars' orbits about the black hole were
    far shorter than any step).  Returns m, r, v with the black hole at index
    0 (q = 1: one more star).  The same seed gives the same stellar positions
    and velocity directions for every q."""
    if rng is None:
        rng = rng_for(5)
    r, v = _plummer_raw(n_stars, rng)
    ms = 1.0 / (n_stars + q)
    m = np.concatenate([[q * ms], np.full(n_stars, ms)])
    r = np.concatenate([np.zeros((1, 3)), r * (3.0 * np.pi / 16.0)])
    v = np.concatenate([np.zeros((1, 3)), v])
    r, v = _to_com_frame(m, r, v)
    U = potential_energy(m, r)
    K = 0.5 * np.sum(m * np.einsum("ij,ij->i", v, v))
    v = v * np.sqrt(-0.5 * U / K)
    return m, r, v


def hierarchical4(ratio=100.0, rng=None):
    """Two equal circular binaries (masses 1/4, separation a_in = 1/ratio) on
    a circular outer orbit of separation 1 (the hierarchical test of Sec. 3.1;
    total mass 1, G = 1, so the outer period is 2 pi).  Orbits are coplanar and
    prograde with random phases; centre of mass at rest.  Returns m, r, v and
    the outer period."""
    if rng is None:
        rng = rng_for(6)
    a_in = 1.0 / ratio
    xo, wo = elements_to_state(1.0, 1.0, 0.0, 0.0, 0.0, 0.0, rng.uniform(0.0, 2.0 * np.pi))
    ph = rng.uniform(0.0, 2.0 * np.pi, 2)
    xi, wi = elements_to_state(0.5, a_in, 0.0, 0.0, 0.0, 0.0, ph)
    m = np.full(4, 0.25)
    cm = [0.5 * xo, -0.5 * xo]
    cv = [0.5 * wo, -0.5 * wo]
    r = np.stack([cm[0] + 0.5 * xi[0], cm[0] - 0.5 * xi[0],
                  cm[1] + 0.5 * xi[1], cm[1] - 0.5 * xi[1]])
    v = np.stack([cv[0] + 0.5 * wi[0], cv[0] - 0.5 * wi[0],
                  cv[1] + 0.5 * wi[1], cv[1] - 0.5 * wi[1]])
    r, v = _to_com_frame(m, r, v)
    return m, r, v, 2.0 * np.pi


def ensemble(n_sys=4096, n_min=3, n_max=64, seed=SEED_BASE + 4):
    """Independent planetary systems in CSR layout.

    Returns offsets [n_sys+1] (int64), m [N], r [N,3], v [N,3], tau [n_sys]."""
    children = np.random.SeedSequence(seed).spawn(n_sys)
    ns = np.random.Generator(np.random.PCG64(seed)).integers(n_min, n_max + 1, n_sys)
    ms, rs, vs, ts = [], [], [], []
    for k in range(n_sys):
        m, r, v, tau = planetary(int(ns[k]) - 1, rng=np.random.Generator(np.random.PCG64(children[k])))
        ms.append(m)
        rs.append(r)
        vs.append(v)
        ts.append(tau)
    offsets = np.zeros(n_sys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(ns)
    return offsets, np.concatenate(ms), np.concatenate(rs), np.concatenate(vs), np.array(ts)


def test_particles(n=1024, rng=None, m_central=1.0):
    """A central mass at rest at the origin plus n-1 massless particles on
    bound orbits (a in [0.5, 4], e in [0, 0.7], isotropic orientation)."""
    if rng is None:
        rng = rng_for(5)
    k = n - 1
    a = 10.0 ** rng.uniform(np.log10(0.5), np.log10(4.0), k)
    e = rng.uniform(0.0, 0.7, k)
    inc = np.arccos(rng.uniform(-1.0, 1.0, k))
    Om, om, M = (rng.uniform(0.0, 2.0 * np.pi, k) for _ in range(3))
    x, w = elements_to_state(m_central, a, e, inc, Om, om, M)
    m = np.concatenate([[m_central], np.zeros(k)])
    r = np.concatenate([np.zeros((1, 3)), x])
    v = np.concatenate([np.zeros((1, 3)), w])
    return m, r, v


def kepler_cases(count=1000, rng=None, kinds=("elliptic", "hyperbolic", "eccentric",
                                              "parabolic", "distant", "long")):
    """Random two-body problems (mu, x0 [n,3], w0 [n,3], tau [n], kind [n]).

    Each state is drawn by picking |x0|, a target semi-major axis (negative for
    hyperbolic orbits) and a random velocity direction; the speed follows from
    the energy.  ``eccentric`` picks radial-ish velocities; ``parabolic`` sets
    the energy within 1e-6 of zero; ``distant`` mimics weakly interacting
    cluster pairs; ``long`` spans several periods."""
    if rng is None:
        rng = rng_for(6)
    per = count // len(kinds)
    out_mu, out_x, out_w, out_t, out_k = [], [], [], [], []
    for kind in kinds:
        n = per
        mu = 10.0 ** rng.uniform(-4.0, 1.0, n)
        r0 = 10.0 ** rng.uniform(-3.0, 1.0, n)
        x = r0[:, None] * _isotropic(rng, n)
        d = _isotropic(rng, n)
        if kind == "elliptic":
            a = r0 * rng.uniform(0.55, 5.0, n)
        elif kind == "hyperbolic":
            a = -r0 * 10.0 ** rng.uniform(-2.0, 2.0, n)
        elif kind == "eccentric":
            a = r0 * rng.uniform(0.5001, 0.6, n)
            rad = x / r0[:, None]
            d = rad + 0.02 * rng.standard_normal((n, 3))
            d /= np.linalg.norm(d, axis=1)[:, None]
        elif kind == "parabolic":
            a = r0 / (1e-6 * rng.uniform(-1.0, 1.0, n))
        elif kind == "distant":
            a = -r0 * 10.0 ** rng.uniform(-4.0, -2.0, n)
        else:  # long: bound orbits over several periods
            a = r0 * rng.uniform(0.55, 2.0, n)
        v2 = mu * (2.0 / r0 - 1.0 / a)
        w = np.sqrt(np.maximum(v2, 0.0))[:, None] * d
        if kind == "long":
            P = 2.0 * np.pi * np.sqrt(np.abs(a) ** 3 / mu)
            tau = P * rng.uniform(1.5, 4.0, n) * rng.choice([-1.0, 1.0], n)
        elif kind == "distant":
            tau = 1e-3 * r0 / np.maximum(np.sqrt(v2), 1e-300) * rng.uniform(0.5, 2.0, n)
        else:
            tdyn = np.sqrt(r0 ** 3 / mu)
            tau = tdyn * 10.0 ** rng.uniform(-3.0, 0.5, n) * rng.choice([-1.0, 1.0], n)
        out_mu.append(mu)
        out_x.append(x)
        out_w.append(w)
        out_t.append(tau)
        out_k += [kind] * n
    return (np.concatenate(out_mu), np.concatenate(out_x), np.concatenate(out_w),
            np.concatenate(out_t), np.array(out_k))


CONFIGS = {
    0: dict(name="planetary N=16, tau=P_in/64", steps=1000),
    1: dict(name="Plummer N=4096, tau=1/1024", steps=64),
    2: dict(name="cluster+BH+binaries N=16384, tau=1/2048", steps=32),
    4: dict(name="ensemble 4096 planetary systems N in [3,64]", steps=256),
}


def config(k):
    """(m, r, v, tau, steps) of the standard workloads 0, 1, 2."""
    if k == 0:
        m, r, v, tau = planetary(15)
    elif k == 1:
        m, r, v, tau = plummer(4096)
    elif k == 2:
        m, r, v, tau = cluster()
    else:
        raise ValueError(k)
    return m, r, v, tau, CONFIGS[k]["steps"]
