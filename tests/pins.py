"""Independent references that pin the oracle (no code shared with it).

* ``kepler_elements``  -- two-body propagation through classical Kepler's
  equation (eccentric or hyperbolic anomaly) in numpy long double.
* ``rk4_nbody``        -- brute-force Newtonian direct integration (classical
  RK4, long double) for small N.
* ``leapfrog_dkd``     -- one drift-kick-drift leapfrog step.
"""
import numpy as np

LD = np.longdouble
PI = LD("3.14159265358979323846264338327950288")


def _solve_monotone(g, dg, lo, hi, iters=200):
    """Root of an increasing function on [lo, hi]: Newton, safeguarded."""
    x = (lo + hi) / 2
    for _ in range(iters):
        gx = g(x)
        if gx == 0:
            return x
        if gx < 0:
            lo = x
        else:
            hi = x
        nx = x - gx / dg(x)
        if not (lo <= nx <= hi):
            nx = (lo + hi) / 2
        if abs(nx - x) <= 4 * np.finfo(LD).eps * max(abs(nx), LD(1e-300)):
            return nx
        x = nx
    return x


def kepler_elements(tau, mu, x0, w0):
    """Relative state after time tau, from Gauss's f and g functions in the
    eccentric (or hyperbolic) anomaly difference.  Returns long-double arrays."""
    x0 = np.asarray(x0, dtype=LD)
    w0 = np.asarray(w0, dtype=LD)
    mu = LD(mu)
    tau = LD(tau)
    r0 = np.sqrt(np.dot(x0, x0))
    v2 = np.dot(w0, w0)
    sig = np.dot(x0, w0)
    a = 1 / (2 / r0 - v2 / mu)
    if a > 0:
        n = np.sqrt(mu / a ** 3)
        ec = 1 - r0 / a
        es = sig / np.sqrt(mu * a)
        M = n * tau
        g = lambda E: E - ec * np.sin(E) + es * (1 - np.cos(E)) - M
        dg = lambda E: 1 - ec * np.cos(E) + es * np.sin(E)
        dE = _solve_monotone(g, dg, M - 3, M + 3)
        s, c = np.sin(dE), np.cos(dE)
        r = a * (1 - ec * c + es * s)
        f = 1 - (a / r0) * (1 - c)
        gg = tau - (dE - s) / n
        fd = -np.sqrt(mu * a) * s / (r * r0)
        gd = 1 - (a / r) * (1 - c)
    else:
        n = np.sqrt(mu / (-a) ** 3)
        ec = 1 - r0 / a
        es = sig / np.sqrt(-mu * a)
        M = n * tau
        g = lambda H: ec * np.sinh(H) + es * (np.cosh(H) - 1) - H - M
        dg = lambda H: ec * np.cosh(H) + es * np.sinh(H) - 1
        span = LD(1)
        while g(span) < 0:
            span *= 2
        while g(-span) > 0:
            span *= 2
        dH = _solve_monotone(g, dg, -span, span)
        s, c = np.sinh(dH), np.cosh(dH)
        r = a * (1 - ec * c - es * s)
        f = 1 - (a / r0) * (1 - c)
        gg = tau - (s - dH) / n
        fd = -np.sqrt(-mu * a) * s / (r * r0)
        gd = 1 - (a / r) * (1 - c)
    return f * x0 + gg * w0, fd * x0 + gd * w0


def accelerations(m, r, G=1.0):
    m = np.asarray(m, dtype=r.dtype)
    d = r[:, None, :] - r[None, :, :]
    d2 = np.einsum("ijk,ijk->ij", d, d)
    np.fill_diagonal(d2, 1)
    inv3 = 1 / (d2 * np.sqrt(d2))
    np.fill_diagonal(inv3, 0)
    return -G * np.einsum("ij,ijk->ik", m[None, :] * inv3, d)


def rk4_nbody(m, r, v, T, nsub, G=1.0):
    """Classical RK4 over [0, T] with nsub equal steps, long double."""
    r = np.asarray(r, dtype=LD).copy()
    v = np.asarray(v, dtype=LD).copy()
    m = np.asarray(m, dtype=LD)
    h = LD(T) / nsub
    Gl = LD(G)
    for _ in range(nsub):
        k1r, k1v = v, accelerations(m, r, Gl)
        k2r, k2v = v + h / 2 * k1v, accelerations(m, r + h / 2 * k1r, Gl)
        k3r, k3v = v + h / 2 * k2v, accelerations(m, r + h / 2 * k2r, Gl)
        k4r, k4v = v + h * k3v, accelerations(m, r + h * k3r, Gl)
        r = r + h / 6 * (k1r + 2 * k2r + 2 * k3r + k4r)
        v = v + h / 6 * (k1v + 2 * k2v + 2 * k3v + k4v)
    return r, v


def leapfrog_dkd(m, r, v, tau, G=1.0):
    """Drift tau/2, kick tau with the Newtonian acceleration, drift tau/2."""
    rh = r + 0.5 * tau * v
    v1 = v + tau * accelerations(np.asarray(m, dtype=np.float64), rh, G)
    return rh + 0.5 * tau * v1, v1
