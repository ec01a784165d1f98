"""The allocation-free entry point (sakura_evolve_noalloc) through the C ABI
against the allocating one (sakura_evolve): the same kernels on the library's
static scratch instead of handle-owned buffers, so the results are equal bit
for bit.  Two calls in a row, the second with a smaller input (the scratch
keeps the first call's contents), on a fresh handle and on one that has
already run other work; sizes beyond the static maximum and the modes it does
not run are refused before any work."""
import numpy as np
import pytest

from paper_1402_3325_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _dev(torch, *arrays):
    return [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
            for a in arrays]


def _both(torch, h, m, r, v, tau, nsteps):
    mt, ra, va = _dev(torch, m, r, v)
    sa = h.evolve_noalloc(mt, ra, va, tau, nsteps, stats=True)
    rb, vb = _dev(torch, r, v)
    sb = h.evolve(mt, rb, vb, tau, nsteps, stats=True)
    torch.cuda.synchronize()
    return (ra, va, sa), (rb, vb, sb)


@pytest.mark.parametrize("warm,strip", [(False, 0), (True, 0), (False, 4)])
def test_noalloc_equals_evolve_two_calls(torch, warm, strip):
    """strip = 4: work items of four tiles along a row in every row, the partial
    sums in that layout's compact order inside the static scratch."""
    from paper_1402_3325_amd.sakura import NOALLOC_MAX_N, Sakura
    h = Sakura(0, row_strip=strip)
    try:
        if warm:  # the handle's own buffers already hold a larger system
            m, r, v, tau = workloads.plummer(5000, rng=np.random.default_rng(3))
            h.evolve(*_dev(torch, m, r, v), tau, 2)
        cases = [workloads.cluster(n_stars=NOALLOC_MAX_N - 1, rng=np.random.default_rng(7)),
                 workloads.plummer(701, rng=np.random.default_rng(8))]
        for k, (m, r, v, tau) in enumerate(cases):
            (ra, va, sa), (rb, vb, sb) = _both(torch, h, m, r, v, tau, 3)
            n = len(m)
            assert torch.equal(ra, rb) and torch.equal(va, vb), (warm, k, n)
            assert sa["pair_solves"] == sb["pair_solves"] == 3 * n * (n - 1) // 2
            assert sa["iters_total"] == sb["iters_total"]
            assert sa["call_ms"] == 0.0 and sa["pair_kernel_ms"] == 0.0
    finally:
        h.close()


def test_noalloc_refuses_what_it_cannot_hold(torch):
    from paper_1402_3325_amd.sakura import (EINVAL, NOALLOC_MAX_N, Sakura, SakuraError,
                                            HARVEST_ROW)
    h = Sakura(0)
    try:
        m, r, v, tau = workloads.plummer(NOALLOC_MAX_N + 1, rng=np.random.default_rng(9))
        mt, rt, vt = _dev(torch, m, r, v)
        with pytest.raises(SakuraError) as e:
            h.evolve_noalloc(mt, rt, vt, tau, 1)
        assert e.value.code == EINVAL
        assert np.array_equal(rt.cpu().numpy(), r)
        rows = torch.zeros((16, HARVEST_ROW), dtype=torch.float32, device="cuda")
        h.harvest_begin(rows, [0.25, 64.0, -1.0, 3.0])
        try:
            m2, r2, v2, tau2 = workloads.plummer(100, rng=np.random.default_rng(10))
            with pytest.raises(SakuraError) as e:
                h.evolve_noalloc(*_dev(torch, m2, r2, v2), tau2, 1)
            assert e.value.code == EINVAL
        finally:
            h.harvest_end()
        # and the entry point works again afterwards
        m3, r3, v3, tau3 = workloads.plummer(130, rng=np.random.default_rng(11))
        (ra, va, _), (rb, vb, _) = _both(torch, h, m3, r3, v3, tau3, 2)
        assert torch.equal(ra, rb) and torch.equal(va, vb)
    finally:
        h.close()


def test_noalloc_matches_oracle(torch, oracle):
    """One step on the static scratch against the oracle (1e-12 per step)."""
    from paper_1402_3325_amd.sakura import Sakura
    from tests.test_gpu_parity import step_error
    m, r, v, tau = workloads.cluster(n_stars=2999, rng=np.random.default_rng(12))
    h = Sakura(0)
    try:
        mt, rt, vt = _dev(torch, m, r, v)
        h.evolve_noalloc(mt, rt, vt, tau, 1)
        torch.cuda.synchronize()
    finally:
        h.close()
    ro, vo = oracle.step(m, r, v, tau)
    er, ev = step_error(rt.cpu().numpy(), vt.cpu().numpy(), ro, vo, r, v)
    assert er <= 1e-12 and ev <= 1e-12, (er, ev)
