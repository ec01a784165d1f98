"""Compositions of the step (Sec. 2.2) on the GPU: sakura_evolve_scheme
against the oracle's schemes, per step from identical inputs (the error metric
and the 1e-12 tolerance of the step parity tests), plus closed-form and
identity checks at full size.

A multi-stage step feeds each stage's output to the next, so the GPU's and the
oracle's rounding differences in one stage's output are inputs to the later
stages.  A tight binary holds its relative state in absolute coordinates only
to ulp(|r|) / a (about 3e-12 for a = 7e-4 at |r| = 6 in the clusters below),
and the Kepler flow over a good part of its period amplifies that further: a
one-ulp difference after the first stage moves the step's result by up to
1e-10.  The per-step comparison therefore allows max(1e-12, 10 S), S the change
of the oracle's own step under a 1e-14 relative perturbation of its input;
the stages themselves are held to 1e-12 by the decomposition test (a triple
jump is three merged steps, bitwise) and the step parity tests."""
import numpy as np
import pytest

from paper_1402_3325_amd import workloads
from tests.test_gpu_parity import TOL, _dev, step_error

pytestmark = pytest.mark.gpu

SCHEMES = {"psi": (0, 1), "unmerged": (1, 2), "triple_jump": (2, 3)}  # (id, stages)


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


def conditioned_tol(oracle, m, r, v, dt, sid, eps=2.0 ** -52, trials=3):
    """(tolerance, oracle result): max(TOL, 10 S), S the largest step error
    between the oracle's step from (r, v) and from (r, v) perturbed by a
    relative eps (one unit in the last place)."""
    ro, vo = oracle.evolve_scheme(m, r, v, dt, 1, sid)
    rng = np.random.default_rng(0)
    sens = 0.0
    for _ in range(trials):
        rp = r * (1.0 + eps * rng.standard_normal(r.shape))
        vp = v * (1.0 + eps * rng.standard_normal(v.shape))
        r2, v2 = oracle.evolve_scheme(m, rp, vp, dt, 1, sid)
        sens = max(sens, *step_error(r2, v2, ro, vo, r, v))
    return max(TOL, 10.0 * sens), (ro, vo)


def triple_jump_weights():
    """g1 = 1/(2 - 2^(1/3)) rounded correctly to double (decimal arithmetic at
    60 digits, then one rounding), g0 = 1 - 2 g1."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 60
        g1 = float(1 / (2 - Decimal(2) ** (Decimal(1) / Decimal(3))))
    return g1, 1.0 - 2.0 * g1


def gpu_scheme(torch, lib, m, r, v, tau, scheme, nsteps=1, stats=False):
    mt, rt, vt = _dev(torch, m, r, v)
    st = lib.evolve_scheme(mt, rt, vt, tau, nsteps, SCHEMES[scheme][0], stats=stats)
    torch.cuda.synchronize()
    return rt.cpu().numpy(), vt.cpu().numpy(), st


@pytest.mark.parametrize("scheme", SCHEMES)
def test_scheme_parity_planetary_every_step(torch, lib, oracle, scheme):
    """Planetary system (N = 16): 12 consecutive steps, each compared from
    the oracle's own state."""
    m, r, v, tau = workloads.planetary(15)
    sid = SCHEMES[scheme][0]
    worst = (0.0, 0.0)
    for _ in range(12):
        rg, vg, _ = gpu_scheme(torch, lib, m, r, v, tau, scheme)
        ro, vo = oracle.evolve_scheme(m, r, v, tau, 1, sid)
        worst = tuple(map(max, worst, step_error(rg, vg, ro, vo, r, v)))
        r, v = ro, vo
    print(scheme, "planetary worst err_r, err_v:", worst)
    assert worst[0] <= TOL and worst[1] <= TOL


@pytest.mark.parametrize("scheme", ["unmerged", "triple_jump"])
def test_scheme_parity_row_strips(torch, oracle, scheme):
    """The stages' pair launches with work items of 4 tiles along a row
    (opts.row_strip; the drift split of eqs. 19a/b runs the kernel that forms
    the increments outside the solver) on 1000 particles, forward and backward
    in time, against the oracle's scheme step."""
    from paper_1402_3325_amd.sakura import Sakura
    m, r, v, tau = workloads.cluster(n_stars=999, rng=np.random.default_rng(2400))
    sid = SCHEMES[scheme][0]
    h = Sakura(0, row_strip=4)
    try:
        for dt in (tau, -2.0 * tau):
            rg, vg, st = gpu_scheme(torch, h, m, r, v, dt, scheme, stats=True)
            assert st["pair_solves"] == SCHEMES[scheme][1] * 1000 * 999 // 2
            tol, (ro, vo) = conditioned_tol(oracle, m, r, v, dt, sid)
            er, ev = step_error(rg, vg, ro, vo, r, v)
            print(scheme, "strips of 4", dt, "err", er, ev, "tol", tol)
            assert er <= tol and ev <= tol, (scheme, dt, er, ev, tol)
    finally:
        h.close()


@pytest.mark.parametrize("scheme", ["unmerged", "triple_jump"])
@pytest.mark.parametrize("n", [2, 3, 65, 333, 1000])
def test_scheme_parity_ragged_sizes(torch, lib, oracle, scheme, n):
    """Sizes around the 64-particle tile with ragged tails, forward and
    backward in time (the triple jump's middle stage runs backward anyway)."""
    rng = np.random.default_rng(2000 + n)
    cases = [workloads.plummer(n, rng=rng)]
    if n >= 3:
        cases.append(workloads.cluster(n_stars=n - 1, rng=rng))
    sid = SCHEMES[scheme][0]
    for m, r, v, tau in cases:
        for dt in (tau, -2.0 * tau):
            rg, vg, _ = gpu_scheme(torch, lib, m, r, v, dt, scheme)
            tol, (ro, vo) = conditioned_tol(oracle, m, r, v, dt, sid)
            er, ev = step_error(rg, vg, ro, vo, r, v)
            print(scheme, n, dt, "err", er, ev, "tol", tol)
            assert er <= tol and ev <= tol, (scheme, n, dt, er, ev, tol)


@pytest.mark.parametrize("n", [3, 65, 1000])
def test_triple_jump_is_three_merged_steps(torch, lib, n):
    """The triple jump's stages are merged steps over g1 dt, g0 dt, g1 dt
    with the drifts between them fused into one kernel: bitwise equal to three
    sakura_evolve calls (each held to the oracle by the step parity tests)."""
    rng = np.random.default_rng(2000 + n)
    m, r, v, tau = workloads.cluster(n_stars=n - 1, rng=rng)
    g1, g0 = triple_jump_weights()
    for dt in (tau, -2.0 * tau):
        rg, vg, _ = gpu_scheme(torch, lib, m, r, v, dt, "triple_jump")
        mt, rt, vt = _dev(torch, m, r, v)
        for g in (g1, g0, g1):
            lib.evolve(mt, rt, vt, g * dt, 1)
        torch.cuda.synchronize()
        assert np.array_equal(rg, rt.cpu().numpy()) and np.array_equal(vg, vt.cpu().numpy())


@pytest.mark.parametrize("scheme", ["unmerged", "triple_jump"])
def test_scheme_parity_plummer_4096(torch, lib, oracle, scheme):
    """Equal-mass Plummer N = 4096 (tau = 1/1024), every particle, one step;
    the pair-solve count is stages x N(N-1)/2."""
    m, r, v, tau, _ = workloads.config(1)
    sid, stages = SCHEMES[scheme]
    rg, vg, st = gpu_scheme(torch, lib, m, r, v, tau, scheme, stats=True)
    ro, vo = oracle.evolve_scheme(m, r, v, tau, 1, sid)
    er, ev = step_error(rg, vg, ro, vo, r, v)
    print(scheme, "plummer4096 err", er, ev)
    assert er <= TOL and ev <= TOL  # no binaries: well conditioned
    assert st["pair_solves"] == stages * (4096 * 4095 // 2)
    assert st["pair_launches"] == stages


@pytest.mark.parametrize("cfg", [1, 2])
def test_unmerged_equals_two_half_steps(torch, lib, cfg):
    """eq. (24) over tau against two eq. (25) steps over tau/2, equal in exact
    arithmetic, on the Plummer sphere (N = 4096, no binaries: to 1e-12) and the
    full-size cluster (N = 16384 with binaries: to max(1e-12, 10 S), S the
    change of the GPU's own unmerged step under a 1e-14 relative perturbation
    of its input)."""
    m, r, v, tau, _ = workloads.config(cfg)
    ru, vu, _ = gpu_scheme(torch, lib, m, r, v, tau, "unmerged")
    rp, vp, _ = gpu_scheme(torch, lib, m, r, v, 0.5 * tau, "psi", nsteps=2)
    er, ev = step_error(ru, vu, rp, vp, r, v)
    tol = TOL
    if cfg == 2:
        rng = np.random.default_rng(0)
        rq, vq, _ = gpu_scheme(torch, lib, m, r * (1.0 + 1e-14 * rng.standard_normal(r.shape)),
                               v * (1.0 + 1e-14 * rng.standard_normal(v.shape)), tau, "unmerged")
        tol = max(TOL, 10.0 * max(step_error(rq, vq, ru, vu, r, v)))
    print("unmerged vs two half steps, config", cfg, ":", er, ev, "tol", tol)
    assert er <= tol and ev <= tol


@pytest.mark.parametrize("scheme", ["unmerged", "triple_jump"])
def test_scheme_massless_particles_16384(torch, lib, scheme):
    """A central mass and 16383 massless particles: every scheme moves each
    particle on its exact Kepler orbit (Gauss's f and g functions)."""
    from tests import pins
    m, r, v = workloads.test_particles(16384)
    tau = 0.05
    rg, vg, _ = gpu_scheme(torch, lib, m, r, v, tau, scheme, nsteps=2)
    rng = np.random.default_rng(5)
    for i in [1, 2, 16383] + rng.choice(np.arange(1, 16384), 40, replace=False).tolist():
        xr, wr = pins.kepler_elements(2 * tau, m[0], r[i] - r[0], v[i] - v[0])
        xr, wr = np.asarray(xr, dtype=np.float64), np.asarray(wr, dtype=np.float64)
        assert np.max(np.abs((rg[i] - rg[0]) - xr)) <= 1e-12 * np.linalg.norm(xr)
        assert np.max(np.abs((vg[i] - vg[0]) - wr)) <= 1e-12 * np.linalg.norm(wr)


def test_unknown_scheme_is_rejected(torch, lib):
    from paper_1402_3325_amd.sakura import SakuraError, EINVAL
    m, r, v, tau = workloads.planetary(3)
    mt, rt, vt = _dev(torch, m, r, v)
    r0 = rt.clone()
    with pytest.raises(SakuraError) as e:
        lib.evolve_scheme(mt, rt, vt, tau, 1, 7)
    assert e.value.code == EINVAL
    assert torch.equal(rt, r0)


@pytest.mark.parametrize("scheme,nsteps", [("psi", 300), ("triple_jump", 200)])
def test_launch_timing_over_many_launches(torch, lib, scheme, nsteps):
    """More pair launches in one call than the ring of timing events holds
    (256): every launch is counted, the summed pair-kernel time is positive and
    within the call's, and timing leaves the results bitwise unchanged."""
    m, r, v, tau = workloads.planetary(65, rng=np.random.default_rng(31))
    rs, vs, st = gpu_scheme(torch, lib, m, r, v, tau, scheme, nsteps=nsteps, stats=True)
    rq, vq, _ = gpu_scheme(torch, lib, m, r, v, tau, scheme, nsteps=nsteps)
    assert st["pair_launches"] == nsteps * SCHEMES[scheme][1]
    assert 0.0 < st["pair_kernel_ms"] <= st["call_ms"]
    assert st["failed_step"] == -1
    assert np.array_equal(rs, rq) and np.array_equal(vs, vq)
