"""Is the pair kernels' summation enough for 1e-12 per step?

Each row of eqs. (27b, 27c) sums N - 1 weighted pair increments.  The tile
kernel adds them in chains of at most 64 terms (one 64 x 64 tile: the i-side
sums in registers, the j-side sums in LDS, both one fused multiply-add per
term); where a work item is a row strip of up to 4 tiles, the strip adds its
tiles' i-side chain results in one more chain of at most 3 additions; and the
partials of a row are combined with TwoSum in a fixed order.  A chain of k
rounded additions errs by at most gamma_k = k u / (1 - k u) times the sum of
the magnitudes it adds (u = 2^-53), and nested chains by gamma of their total
depth; the compensated combination adds 2 u |S| plus terms of order nb^2 u^2,
so a row's summation error is below gamma_67 sum_j |t_j| + 2 u |S|, against
gamma_(N-1) sum_j |t_j| for one flat chain of N - 1 terms.

The first test evaluates both bounds on the benchmark cluster (N = 16384) from
the oracle's own increments, for the central mass, the members of the
tightest binaries and random stars, in the per-step error metric: the blocked
bound stays below 2e-14 everywhere, while the flat one exceeds 1e-12 for
binary members (their companion's increment is of the size of their velocity,
so N u of it is not small).  The second emulates the two orders on a
constructed worst case and checks each against the exact sum (math.fsum)."""
import math

import numpy as np

from paper_1402_3325_amd import workloads

U = 2.0 ** -53


def gamma(k):
    return k * U / (1.0 - k * U)


def test_blocked_bound_holds_on_the_benchmark_cluster(oracle):
    from scipy.spatial import cKDTree
    m, r, v, tau, _ = workloads.config(2)
    n = len(m)
    d, j = cKDTree(r[1:]).query(r[1:], k=2)
    tight = np.argsort(d[:, 1])[:8] + 1
    rows = sorted({0, *tight.tolist(), *(j[tight - 1, 1] + 1).tolist(),
                   *np.random.default_rng(1).choice(n, 16, replace=False).tolist()})
    r_rms = np.sqrt(np.mean(np.sum(r ** 2, 1)))
    v_rms = np.sqrt(np.mean(np.sum(v ** 2, 1)))
    worst_blocked = worst_flat = 0.0
    for i in rows:
        dr, dv = oracle.row_terms(m, r, v, tau, i)
        for t, scale in ((dr, max(np.linalg.norm(r[i]), r_rms)),
                         (dv, max(np.linalg.norm(v[i]), v_rms))):
            A = np.abs(t).sum(0)
            S = np.abs(t.sum(0))
            blocked = float(np.max(gamma(64 + 3) * A + 2.0 * U * S)) / scale
            flat = float(np.max(gamma(n - 1) * A)) / scale
            worst_blocked = max(worst_blocked, blocked)
            worst_flat = max(worst_flat, flat)
    print(f"row summation bounds, per-step metric: blocked {worst_blocked:.2e}, "
          f"flat {worst_flat:.2e}")
    assert worst_blocked <= 2e-14
    assert worst_flat > 1e-12  # a flat chain would not be guaranteed


def _kernel_order_sum(t, tile=64, strip=1):
    """The tile kernel's order on one row's terms: chains of `tile` rounded
    additions; the chain results of `strip` consecutive tiles added in one
    more chain (a row strip's i side); then TwoSum over those in order, and
    s + e."""
    chains = []
    for a in range(0, len(t), tile):
        acc = 0.0
        for x in t[a:a + tile]:
            acc = acc + float(x)
        chains.append(acc)
    parts = []
    for a in range(0, len(chains), strip):
        acc = chains[a]
        for x in chains[a + 1:a + strip]:
            acc = acc + x
        parts.append(acc)
    s = e = 0.0
    for x in parts:
        y = s + x
        bp = y - s
        e += (s - (y - bp)) + (x - bp)
        s = y
    return s + e


def _flat_sum(t):
    acc = 0.0
    for x in t:
        acc = acc + float(x)
    return acc


def test_blocked_order_holds_where_a_flat_chain_fails():
    """A large term followed by N - 2 terms of 0.75 ulp of it (each addition
    to the running sum rounds the same way) and its negative at the end: the
    flat chain errs by about (N - 2) / 4 ulp, the kernel's order only within
    the first and last chain."""
    n = 16384
    A = 1.0
    t = np.full(n, 0.75 * math.ulp(A))
    t[0] = A
    t[-1] = -A
    exact = math.fsum(t.tolist())
    scale = 0.5 * A  # a velocity scale of the order of the large increment
    e_flat = abs(_flat_sum(t) - exact) / scale
    assert e_flat > 1e-12
    for strip in (1, 4):
        e_blocked = abs(_kernel_order_sum(t, strip=strip) - exact) / scale
        print(f"constructed worst case: flat {e_flat:.2e}, kernel order with strips of "
              f"{strip}: {e_blocked:.2e}")
        assert e_blocked <= 2.0 * gamma(64 + strip - 1) * (2 * A) / scale
        assert e_blocked <= 1e-13
