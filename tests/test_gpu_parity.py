"""GPU (HIP library through the C ABI) vs the CPU oracle, per step from
identical inputs.

Error metric, for positions (velocities alike):
    err_r = max_i |r_gpu,i - r_ref,i| / max(|r_ref,i|, r_rms)
with r_rms the root-mean-square |r| of the input state.  Comparing a single
step from identical inputs keeps the chaotic growth of differences out of the
measure.  Tolerance: 1e-12 (relative) on positions and velocities per step.
"""
import numpy as np
import pytest

from paper_1402_3325_amd import workloads
from tests import pins

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def lib(torch):
    from paper_1402_3325_amd.sakura import Sakura
    h = Sakura(0)
    yield h
    h.close()


def _dev(torch, *arrays):
    return [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda") for a in arrays]


def gpu_step(torch, lib, m, r, v, tau, G=1.0, nsteps=1, stats=False):
    mt, rt, vt = _dev(torch, m, r, v)
    st = lib.evolve(mt, rt, vt, tau, nsteps, G=G, stats=stats)
    torch.cuda.synchronize()
    return rt.cpu().numpy(), vt.cpu().numpy(), st


def step_error(r_out, v_out, r_ref, v_ref, r_in, v_in):
    r_rms = np.sqrt(np.mean(np.sum(r_in ** 2, axis=1)))
    v_rms = np.sqrt(np.mean(np.sum(v_in ** 2, axis=1)))
    er = np.linalg.norm(r_out - r_ref, axis=1) / np.maximum(np.linalg.norm(r_ref, axis=1), r_rms)
    ev = np.linalg.norm(v_out - v_ref, axis=1) / np.maximum(np.linalg.norm(v_ref, axis=1), v_rms)
    return float(er.max()), float(ev.max())


def test_parity_planetary_every_step(torch, lib, oracle):
    """Planetary system (N = 16, tau = P_in/64): 25 consecutive steps, each
    compared from the oracle's own state."""
    m, r, v, tau = workloads.planetary(15)
    worst = (0.0, 0.0)
    for _ in range(25):
        rg, vg, _ = gpu_step(torch, lib, m, r, v, tau)
        ro, vo = oracle.step(m, r, v, tau)
        e = step_error(rg, vg, ro, vo, r, v)
        worst = tuple(map(max, worst, e))
        r, v = ro, vo
    print("planetary worst err_r, err_v:", worst)
    assert worst[0] <= TOL and worst[1] <= TOL


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 130, 200, 333])
def test_parity_ragged_sizes(torch, lib, oracle, n):
    """Sizes below, at and past the 64-particle tile, with ragged tails; a
    Plummer sphere and a cluster with a central mass and binaries."""
    rng = np.random.default_rng(1000 + n)
    cases = [workloads.plummer(n, rng=rng)]
    if n >= 3:
        cases.append(workloads.cluster(n_stars=n - 1, rng=rng))
    for m, r, v, tau in cases:
        for dt in (tau, -3.0 * tau):
            rg, vg, _ = gpu_step(torch, lib, m, r, v, dt)
            ro, vo = oracle.step(m, r, v, dt)
            er, ev = step_error(rg, vg, ro, vo, r, v)
            assert er <= TOL and ev <= TOL, (n, dt, er, ev)


def test_parity_plummer_4096_full(torch, lib, oracle):
    """Equal-mass Plummer N = 4096 (tau = 1/1024): every particle, 3 steps."""
    m, r, v, tau, _ = workloads.config(1)
    for _ in range(3):
        rg, vg, st = gpu_step(torch, lib, m, r, v, tau, stats=True)
        ro, vo = oracle.step(m, r, v, tau)
        er, ev = step_error(rg, vg, ro, vo, r, v)
        print("plummer4096 err", er, ev, "mean iters", st["iters_total"] / st["pair_solves"])
        assert er <= TOL and ev <= TOL
        assert st["pair_solves"] == 4096 * 4095 // 2
        r, v = ro, vo


@pytest.mark.parametrize("n", [1000, 6000, 9000])
def test_parity_split_tiles(torch, lib, oracle, n):
    """Where the tiles alone would leave most wave slots of the device empty,
    each tile's sub-steps are split over 2 or 4 wavefronts (on 256 compute
    units: 4 at n = 1000, 2 at n = 6000, 1 at n = 9000).  Every row against
    the oracle; the exact number of pair solves; and the diagnostic copy, which
    splits alike, bitwise equal, with its per-pair histogram matching the
    packed counters."""
    from paper_1402_3325_amd.sakura import Sakura
    m, r, v, tau = workloads.cluster(n_stars=n - 1, rng=np.random.default_rng(7000 + n))
    rg, vg, st = gpu_step(torch, lib, m, r, v, tau, stats=True)
    ro, vo = oracle.step(m, r, v, tau)
    er, ev = step_error(rg, vg, ro, vo, r, v)
    print(f"n={n} err {er:.2e} {ev:.2e}")
    assert er <= TOL and ev <= TOL
    assert st["pair_solves"] == n * (n - 1) // 2
    hd = Sakura(0, histogram=True)
    try:
        rd, vd, sd = gpu_step(torch, hd, m, r, v, tau, stats=True)
    finally:
        hd.close()
    hist = np.array(sd["hist"], dtype=np.int64)
    assert np.array_equal(rd, rg) and np.array_equal(vd, vg)
    assert sd["pair_solves"] == st["pair_solves"] == hist.sum()
    assert sd["iters_total"] == st["iters_total"] == int(np.sum(np.arange(32) * hist))
    assert sd["iters_max"] == st["iters_max"]


@pytest.mark.parametrize("n", [1000, 3000])
def test_parity_row_strips(torch, oracle, n):
    """Work items of S tiles along a row of the upper triangle (opts.row_strip,
    one wavefront per tile), the i-side partial sums written once per item and
    stored compactly: S = 2, 4, 8 and S past the number of blocks (every row
    one strip, the diagonal tile first), on 16 and 47 blocks with a ragged last
    block.  Every
    row against the oracle; the exact pair-solve count; the results of
    different S within rounding of each other (the partial sums are grouped
    differently); the diagnostic copy with the same S bitwise equal."""
    from paper_1402_3325_amd.sakura import Sakura
    m, r, v, tau = workloads.cluster(n_stars=n - 1, rng=np.random.default_rng(7100 + n))
    ro, vo = oracle.step(m, r, v, tau)
    outs = {}
    for S in (1, 2, 4, 8, 64):
        h = Sakura(0, row_strip=S)
        try:
            rg, vg, st = gpu_step(torch, h, m, r, v, tau, stats=True)
        finally:
            h.close()
        er, ev = step_error(rg, vg, ro, vo, r, v)
        print(f"n={n} S={S} err {er:.2e} {ev:.2e}", flush=True)
        assert er <= TOL and ev <= TOL, (S, er, ev)
        assert st["pair_solves"] == n * (n - 1) // 2
        outs[S] = (rg, vg, st)
    for S in (2, 4, 8, 64):
        e = step_error(outs[S][0], outs[S][1], outs[1][0], outs[1][1], r, v)
        assert max(e) <= 1e-14, (S, e)
        assert outs[S][2]["iters_total"] == outs[1][2]["iters_total"]
    hd = Sakura(0, histogram=True, row_strip=4)
    try:
        rd, vd, sd = gpu_step(torch, hd, m, r, v, tau, stats=True)
    finally:
        hd.close()
    assert np.array_equal(rd, outs[4][0]) and np.array_equal(vd, outs[4][1])
    assert sd["pair_solves"] == int(np.sum(sd["hist"]))


def test_parity_default_strips_ragged(torch, lib, oracle):
    """The default layout where it splits: n = 12345 (193 blocks, the last one
    holding 57 particles) runs strips of 4 tiles in the rows of blocks 0..64
    and single tiles in the triangle of the last 128 blocks on 256 compute
    units; every row against the oracle's step, the exact pair-solve count, and
    the same step with one tile per item (row_strip = 1) within rounding."""
    from paper_1402_3325_amd.sakura import Sakura
    n = 12345
    m, r, v, tau = workloads.cluster(n_stars=n - 1, rng=np.random.default_rng(7300))
    rg, vg, st = gpu_step(torch, lib, m, r, v, tau, stats=True)
    assert st["pair_solves"] == n * (n - 1) // 2
    ro, vo = oracle.step(m, r, v, tau)
    er, ev = step_error(rg, vg, ro, vo, r, v)
    print(f"n={n} default layout err {er:.2e} {ev:.2e}", flush=True)
    assert er <= TOL and ev <= TOL
    h1 = Sakura(0, row_strip=1)
    try:
        r1, v1, s1 = gpu_step(torch, h1, m, r, v, tau, stats=True)
    finally:
        h1.close()
    assert s1["iters_total"] == st["iters_total"]
    assert max(step_error(rg, vg, r1, v1, r, v)) <= 1e-14


def _cluster_rows(m, r, rng, count=64, tight=32):
    """Rows to sample in a cluster: the central mass (row 0), the `tight`
    stars closest to a neighbour (members of the tightest binaries) with those
    neighbours, and `count` random stars."""
    from scipy.spatial import cKDTree
    n = len(m)
    d, j = cKDTree(r[1:]).query(r[1:], k=2)  # the nearest star other than itself
    nn_d, nn_j = d[:, 1], j[:, 1] + 1
    rows = {0}
    for i in np.argsort(nn_d)[:tight]:
        rows.update((int(i) + 1, int(nn_j[i])))
    rows.update(rng.choice(n, count, replace=False).tolist())
    return np.array(sorted(rows), dtype=np.int64)


def test_parity_cluster_16384_every_row(torch, lib, oracle):
    """Full-size cluster (N = 16384, central mass, 10 % binaries,
    tau = 1/2048) in the benchmark's launch configuration (sakura_evolve):
    every particle compared with the full oracle step, over two steps (the
    second from the oracle's own state)."""
    m, r, v, tau, _ = workloads.config(2)
    rin, vin = r, v
    for step in range(2):
        rg, vg, st = gpu_step(torch, lib, m, rin, vin, tau, stats=True)
        assert st["pair_solves"] == 16384 * 16383 // 2
        ro, vo = oracle.step(m, rin, vin, tau)
        er, ev = step_error(rg, vg, ro, vo, rin, vin)
        print("cluster16384 step", step, "err", er, ev, "iters mean",
              st["iters_total"] / st["pair_solves"], "max", st["iters_max"], flush=True)
        assert er <= TOL and ev <= TOL
        rin, vin = ro, vo


def test_boundary_rejects_invalid_arguments(torch, lib):
    """n < 2, G <= 0 or not finite, a tile override outside [0, 64], a model
    blob of the wrong size, and n whose partial sums exceed the device: EINVAL
    before any work, with the caller's arrays untouched."""
    from paper_1402_3325_amd.sakura import Sakura, SakuraError, EINVAL
    import ctypes
    m1, r1, v1 = _dev(torch, np.array([0.7]), np.array([[0.1, 0.2, 0.3]]),
                      np.array([[1.0, -2.0, 0.5]]))
    with pytest.raises(SakuraError) as e:
        lib.evolve(m1, r1, v1, 0.01, 1)
    assert e.value.code == EINVAL
    m, r, v, tau = workloads.plummer(70, rng=np.random.default_rng(3))
    mt, rt, vt = _dev(torch, m, r, v)
    for G in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(SakuraError) as e:
            lib.evolve(mt, rt, vt, tau, 1, G=G)
        assert e.value.code == EINVAL
        with pytest.raises(SakuraError) as e:
            lib.energy(mt, rt, vt, G=G)
        assert e.value.code == EINVAL
    assert np.array_equal(rt.cpu().numpy(), r) and np.array_equal(vt.cpu().numpy(), v)
    for bad in (-1, 65):
        with pytest.raises(SakuraError) as e:
            Sakura(0, tile_override=bad)
        assert e.value.code == EINVAL
    for bad in (-1, 3, 65, 128):
        with pytest.raises(SakuraError) as e:
            Sakura(0, row_strip=bad)
        assert e.value.code == EINVAL
    blob = (ctypes.c_char * 64)()
    assert lib._lib.sakura_set_guess_model(lib._h, ctypes.cast(blob, ctypes.c_void_p), 64) == EINVAL
    # 2^20 particles would need 0.5 TB of partial sums (0.8 TB with one tile per item)
    n = 1 << 20
    mb = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
    rb = torch.rand((n, 3), dtype=torch.float64, device="cuda")
    vb = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    r_before = rb.clone()
    with pytest.raises(SakuraError) as e:
        lib.evolve(mb, rb, vb, 1e-3, 1)
    assert e.value.code == EINVAL and "partial sums" in str(e.value)
    assert torch.equal(rb, r_before)


def test_max_rel_residual_in_diagnostic_mode(torch, oracle):
    """With opts.histogram the pair kernels evaluate the Kepler equation once
    more at every accepted root: the largest relative residual |t(s) - t|/|t|
    is at the rounding level of t(s) (a few ulps); without it the field is 0.
    The results are the same either way, bit for bit."""
    from paper_1402_3325_amd.sakura import Sakura
    m, r, v, tau = workloads.cluster(n_stars=4095, rng=np.random.default_rng(12))
    hd, hp = Sakura(0, histogram=True), Sakura(0)
    try:
        rd, vd, sd = gpu_step(torch, hd, m, r, v, tau, stats=True)
        rp, vp, sp = gpu_step(torch, hp, m, r, v, tau, stats=True)
    finally:
        hd.close()
        hp.close()
    print("max relative residual", sd["max_rel_residual"])
    assert 0.0 < sd["max_rel_residual"] <= 1e-13
    assert sp["max_rel_residual"] == 0.0
    assert np.array_equal(rd, rp) and np.array_equal(vd, vp)


def test_massless_particles_exact_orbits_16384(torch, lib):
    """A central mass and 16383 massless particles: every particle follows its
    exact Kepler orbit (closed form in long double), at full size."""
    m, r, v = workloads.test_particles(16384)
    tau = 0.01
    rg, vg, _ = gpu_step(torch, lib, m, r, v, tau, nsteps=4)
    assert np.array_equal(vg[0], v[0]) and np.allclose(rg[0], r[0] + 4 * tau * v[0], atol=0)
    rng = np.random.default_rng(3)
    for i in rng.choice(np.arange(1, 16384), 200, replace=False):
        xr, wr = pins.kepler_elements(4 * tau, m[0], r[i] - r[0], v[i] - v[0])
        ex = float(np.max(np.abs((rg[i] - rg[0]) - xr))) / np.linalg.norm(r[i])
        ew = float(np.max(np.abs((vg[i] - vg[0]) - wr))) / np.linalg.norm(v[i])
        assert ex <= TOL and ew <= TOL, (i, ex, ew)


def test_evolve_is_repeated_step_and_deterministic(torch, lib):
    m, r, v, tau = workloads.plummer(300, rng=np.random.default_rng(77))
    r5, v5, _ = gpu_step(torch, lib, m, r, v, tau, nsteps=5)
    r5b, v5b, _ = gpu_step(torch, lib, m, r, v, tau, nsteps=5)
    assert np.array_equal(r5, r5b) and np.array_equal(v5, v5b)
    rr, vv = r, v
    for _ in range(5):
        rr, vv, _ = gpu_step(torch, lib, m, rr, vv, tau)
    assert np.array_equal(rr, r5) and np.array_equal(vv, v5)


def test_two_body_reversal(torch, lib):
    m = np.array([0.7, 0.3])
    r = np.array([[0.3, 0.1, -0.2], [-0.4, 0.2, 0.1]])
    v = np.array([[0.1, 0.9, 0.0], [-0.3, -1.2, 0.2]])
    r1, v1, _ = gpu_step(torch, lib, m, r, v, 0.05)
    r2, v2, _ = gpu_step(torch, lib, m, r1, v1, -0.05)
    assert np.max(np.abs(r2 - r)) <= 1e-14 and np.max(np.abs(v2 - v)) <= 1e-14


def test_massless_system_drifts(torch, lib):
    rng = np.random.default_rng(4)
    m = np.zeros(70)
    r = rng.normal(size=(70, 3))
    v = rng.normal(size=(70, 3))
    rg, vg, st = gpu_step(torch, lib, m, r, v, 0.1, stats=True)
    assert st["pair_solves"] == 0
    assert np.array_equal(vg, v)
    assert np.allclose(rg, r + 0.1 * v, rtol=0, atol=1e-15)


def test_errors_leave_state_unchanged(torch, lib):
    from paper_1402_3325_amd.sakura import SakuraError, ECOLLIDE, ENONFINITE, EINVAL
    m, r, v, tau = workloads.plummer(100, rng=np.random.default_rng(2))
    bad = {}
    rc = r.copy()
    rc[17] = rc[3]
    vc = v.copy()
    vc[17] = vc[3]
    bad[ECOLLIDE] = (m, rc, vc)
    rn = r.copy()
    rn[50, 1] = np.nan
    bad[ENONFINITE] = (m, rn, v)
    mn = m.copy()
    mn[9] = -1.0
    bad[EINVAL] = (mn, r, v)
    for code, (mm, rr, vv) in bad.items():
        mt, rt, vt = _dev(torch, mm, rr, vv)
        with pytest.raises(SakuraError) as e:
            lib.evolve(mt, rt, vt, tau, 3)
        assert e.value.code == code
        out_r, out_v = rt.cpu().numpy(), vt.cpu().numpy()
        assert np.array_equal(out_r, rr, equal_nan=True) and np.array_equal(out_v, vv)
    mt, rt, vt = _dev(torch, m, r, v)
    with pytest.raises(SakuraError):
        lib.evolve(mt, rt, vt, float("nan"), 1)
    # the handle still works after errors
    lib.evolve(mt, rt, vt, tau, 1)


def test_energy_matches_oracle(torch, lib, oracle):
    for k in (0, 1, 2):
        m, r, v, tau, _ = workloads.config(k)
        mt, rt, vt = _dev(torch, m, r, v)
        eg = lib.energy(mt, rt, vt)
        eo = oracle.energy(m, r, v)
        assert abs(eg["E"] - eo["E"]) <= 1e-13 * abs(eo["U"])
        assert abs(eg["K"] - eo["K"]) <= 1e-14 * eo["K"]
        for key in ("P", "L", "Rcm"):
            assert np.max(np.abs(np.array(eg[key]) - eo[key])) <= 1e-14 * (1 + np.abs(eo[key]).max())


def test_counters_agree_with_histogram(torch):
    """The pair kernel's per-lane packed counters (evaluations, safeguarded
    steps, solved pairs) against the exact number of pairs and the per-pair
    histogram, which the kernel counts independently in LDS."""
    from paper_1402_3325_amd.sakura import Sakura
    m, r, v, tau = workloads.cluster()  # N = 16384: some pairs need two or more evaluations
    m2, r2, v2, _ = workloads.plummer(333, rng=np.random.default_rng(8))
    m2 = m2.copy()
    m2[::7] = 0.0  # pairs of two massless particles are not solved
    hh, hp = Sakura(0, histogram=True), Sakura(0)
    try:
        for mm, rr, vv, dt in ((m, r, v, tau), (m2, r2, v2, 0.05)):
            n, nz = len(mm), int(np.sum(mm == 0.0))
            pairs = n * (n - 1) // 2 - nz * (nz - 1) // 2
            st_h = hh.evolve(*_dev(torch, mm, rr, vv), dt, 1, stats=True)
            st_p = hp.evolve(*_dev(torch, mm, rr, vv), dt, 1, stats=True)
            hist = np.array(st_h["hist"], dtype=np.int64)
            assert hist[31] == 0 and hist[0] == 0
            assert st_h["pair_solves"] == st_p["pair_solves"] == pairs == hist.sum()
            assert st_h["iters_total"] == st_p["iters_total"] == int(np.sum(np.arange(32) * hist))
            assert st_h["iters_max"] == st_p["iters_max"] == int(np.nonzero(hist)[0].max())
            assert st_h["fallbacks"] == st_p["fallbacks"]
            assert st_p["iters_total"] > st_p["pair_solves"]  # not only one-evaluation pairs
    finally:
        hh.close()
        hp.close()


def test_max_iter_limit(torch):
    from paper_1402_3325_amd.sakura import Sakura, SakuraError, EINVAL
    with pytest.raises(SakuraError) as e:
        Sakura(0, max_iter=1001)
    assert e.value.code == EINVAL
    h = Sakura(0, max_iter=1000)
    h.close()


@pytest.mark.parametrize("strip", [0, 4])
def test_default_parameters_kernel_matches_general(torch, lib, strip):
    """The tile kernel built for the default solver parameters and the general
    one (any other max_iter) do the same arithmetic: identical results, with
    the default layout (tiles split over wavefronts at this size) and with
    strips of 4 tiles in every row (the general kernel's strip loop)."""
    from paper_1402_3325_amd.sakura import Sakura
    m, r, v, tau = workloads.plummer(4096, rng=np.random.default_rng(5))
    hd = Sakura(0, row_strip=strip) if strip else lib
    hg = Sakura(0, max_iter=41, row_strip=strip)
    try:
        ra, va, sa = gpu_step(torch, hd, m, r, v, tau, nsteps=2, stats=True)
        rb, vb, sb = gpu_step(torch, hg, m, r, v, tau, nsteps=2, stats=True)
    finally:
        hg.close()
        if strip:
            hd.close()
    assert np.array_equal(ra, rb) and np.array_equal(va, vb)
    assert sa["iters_total"] == sb["iters_total"] and sa["pair_solves"] == sb["pair_solves"]
