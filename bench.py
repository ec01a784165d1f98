"""Benchmark: Kepler pair-solves/s of the Sakura step at N = 16384 (FP64).

Workload: a star cluster of 16383 Plummer stars (total mass 1, 10 % in
primordial binaries with a log-uniform in [1e-4, 1e-2] and thermal
eccentricities) around a central point mass 0.01, tau = 1/2048.  One "step" is
one full pass of eqs. (27a-d): the half drifts and all N(N-1)/2 pair solves
with their weighted two-sided sums.  The timed region is one sakura_evolve call
of K steps with the state already resident in HBM.

Prints one JSON line (see the fields below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Kepler pair-solves/s at N=16384 (FP64), learned-guess vs plain at 1e-12 error"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk

# Algorithmic FP64 work per pair solve, the model of the method's cost (fma
# counted as 2): set-up, starter, coefficients, increments and the two-sided
# compensated sums 160 flops, and 70 flops per evaluation of the Kepler
# equation (Stumpff series, residual and derivatives, Laguerre step), so
# F_pair = 160 + 70 k with k the mean number of evaluations per solve, which
# the kernel counts.  `achieved` in the roofline is F_pair x N(N-1)/2 per
# launch over the launch's duration.
FLOPS_SETUP = 160
FLOPS_PER_ITER = 70
# The same work counted in the kernel source along the path almost every pair
# takes (one evaluation in the cheapest tier, accepted by its error bound):
# pair set-up and back-drift 18, Kepler set-up, starter and tier choice 42, the
# evaluation with its Newton or Halley step, tests and shift 52, Lagrange coefficients
# 12, increments, weights and the two-sided sums 46; 92 per further evaluation.
KERNEL_FLOPS_FIRST = 18 + 42 + 52 + 12 + 46
KERNEL_FLOPS_PER_EXTRA_ITER = 92
KERNEL_SOURCES = ["paper_1402_3325_amd/csrc/kepler_device.hpp",
                  "paper_1402_3325_amd/csrc/guess_device.hpp",
                  "paper_1402_3325_amd/csrc/common.hpp",
                  "paper_1402_3325_amd/csrc/tiles.hpp",
                  "paper_1402_3325_amd/csrc/sakura.hip"]
# domain of the learned starter: tau' in [0.25, 64], b' >= -1, |e'| <= 3 (pairs the
# plain starter needs three or more Kepler evaluations for)
GUESS_DOMAIN = [0.25, 64.0, -1.0, 3.0]
LEARNED_REPEATS = 3  # alternating plain / learned timed runs in the learned comparison
PLUMMER_HARVEST_STEPS = 2000  # harvest steps of the independent N = 4096 Plummer sphere
TRAFFIC_FILE = "profiles/k_pairs_cluster16384.traffic.json"


def progress(msg):
    """One line on stderr when a part of the benchmark ends (stdout carries
    only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_profile():
    """The committed rocprofv3 counter record of the pair kernel (HBM bytes
    per launch, clock, hardware FP64 operations per pair), or None when the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def flops_per_pair(mean_iters):
    """The method's algorithmic flops per pair solve (model above)."""
    return FLOPS_SETUP + FLOPS_PER_ITER * mean_iters


def kernel_flops_per_pair(mean_iters):
    return KERNEL_FLOPS_FIRST + KERNEL_FLOPS_PER_EXTRA_ITER * max(mean_iters - 1.0, 0.0)


def step_error(rg, vg, ro, vo, r, v):
    """Per-step error metric over every row: max_i |dr_i| / max(|r_i|, r_rms)
    and the same for velocities."""
    r_rms = np.sqrt(np.mean(np.sum(r ** 2, 1)))
    v_rms = np.sqrt(np.mean(np.sum(v ** 2, 1)))
    er = np.max(np.linalg.norm(rg - ro, axis=1) / np.maximum(np.linalg.norm(ro, axis=1), r_rms))
    ev = np.max(np.linalg.norm(vg - vo, axis=1) / np.maximum(np.linalg.norm(vo, axis=1), v_rms))
    return float(er), float(ev)


def gpu_one_step(lib, torch, m, r, v, tau):
    mt, rt, vt = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (m, r, v))
    st = lib.evolve(mt, rt, vt, tau, 1, stats=True)
    return rt.cpu().numpy(), vt.cpu().numpy(), st


def batched(lib, torch, steps=256):
    """The batched ensemble: 4096 planetary systems with n uniform in
    [3, 64], each with its own tau = innermost period / 64, all systems
    advanced `steps` steps by one sakura_batch_evolve call (one persistent,
    graph-captured launch).  The packing policy is autotuned first."""
    import oracle
    from paper_1402_3325_amd import workloads
    off, m, r, v, tau = workloads.ensemble()
    sizes = np.diff(off)
    pairs = int(np.sum(sizes * (sizes - 1) // 2))
    mt, rt, vt, dt = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (m, r, v, tau))
    best_probe = lib.autotune_batch(off, mt, rt, vt, dt, probe_steps=8)
    # per-step error of one step on sampled systems
    r1, v1 = rt.clone(), vt.clone()
    lib.batch_evolve(off, mt, r1, v1, dt, 1)
    rg, vg = r1.cpu().numpy(), v1.cpu().numpy()
    worst = [0.0, 0.0]
    for k in np.random.default_rng(3).choice(len(sizes), 32, replace=False):
        a, b = off[k], off[k + 1]
        ro, vo = oracle.step(m[a:b], r[a:b], v[a:b], tau[k])
        r_rms = np.sqrt(np.mean(np.sum(r[a:b] ** 2, 1)))
        v_rms = np.sqrt(np.mean(np.sum(v[a:b] ** 2, 1)))
        worst[0] = max(worst[0], float(np.max(np.linalg.norm(rg[a:b] - ro, axis=1) /
                                               np.maximum(np.linalg.norm(ro, axis=1), r_rms))))
        worst[1] = max(worst[1], float(np.max(np.linalg.norm(vg[a:b] - vo, axis=1) /
                                               np.maximum(np.linalg.norm(vo, axis=1), v_rms))))
    # warm-up with the timed call's arguments: the launch sequence is captured
    # into a graph once for them (the step count is one of the arguments it
    # bakes in), and the timed call replays it
    lib.batch_evolve(off, mt, rt, vt, dt, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = lib.batch_evolve(off, mt, rt, vt, dt, steps, stats=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"value": pairs * steps / wall, "unit": "pair-solves/s",
            "workload": "4096 planetary systems, n uniform in [3,64], tau = P_in/64, "
                        f"{steps} steps in one launch",
            "systems": int(len(sizes)), "pairs_per_step": pairs, "steps": steps,
            "ms_total": wall * 1e3, "kernel_ms_events": st["call_ms"],
            "mean_kepler_iters": st["iters_total"] / max(st["pair_solves"], 1),
            "autotune_probe_ms": best_probe,
            "err_vs_oracle": {"err_r": worst[0], "err_v": worst[1], "systems": 32,
                              "tol": 1e-12}}


def plummer4096(lib, torch, steps=64, warmup=16):
    """The equal-mass Plummer sphere of N = 4096 (tau = 1/1024, 64 steps): the
    smaller single-system workload, where the tile kernel splits each tile's
    sub-steps over several wavefronts to fill the device.  Its first step is
    compared with the oracle's over every row."""
    import oracle
    from paper_1402_3325_amd import workloads
    m, r, v, tau, _ = workloads.config(1)
    n = len(m)
    pairs = n * (n - 1) // 2
    mt, rt, vt = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (m, r, v))
    r1, v1 = rt.clone(), vt.clone()
    lib.evolve(mt, r1, v1, tau, 1)
    ro, vo = oracle.step(m, r, v, tau)
    er, ev = step_error(r1.cpu().numpy(), v1.cpu().numpy(), ro, vo, r, v)
    lib.evolve(mt, rt, vt, tau, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = lib.evolve(mt, rt, vt, tau, steps, stats=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pair_ms = st["pair_kernel_ms"] / max(st["pair_launches"], 1)
    return {"value": pairs * steps / wall, "unit": "pair-solves/s",
            "workload": f"Plummer sphere N={n}, tau=1/1024, {steps} steps",
            "ms_per_step": wall * 1e3 / steps, "pair_kernel_ms": pair_ms,
            "kernel_rate": pairs / (pair_ms * 1e-3),
            "mean_kepler_iters": st["iters_total"] / max(st["pair_solves"], 1),
            "err_vs_oracle": {"err_r": er, "err_v": ev, "rows": int(n), "tol": 1e-12}}


def learned(torch, m, r, v, tau, steps, warmup, harvest_steps, oracle_step=None):
    """The learned Kepler starter on the same workload.  Rows are harvested
    with the plain starter from independent runs of the Plummer sphere and of
    the cluster (seed offset 100), the network is trained by the library's own
    kernels, then the timed run of the main workload is repeated with the
    network's starter.  Also reports, for the pairs in the network's domain,
    the Kepler evaluations and the largest final residual of the Kepler
    equation with and without it, the step's error against the oracle over
    every row, and the batched ensemble with the network."""
    from paper_1402_3325_amd import workloads
    from paper_1402_3325_amd.sakura import Sakura, GUESS_ANALYTIC, GUESS_LEARNED
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    h = Sakura(0)
    cap = 12_000_000
    rows = torch.zeros((cap, 12), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    h.harvest_begin(rows, GUESS_DOMAIN)
    m1, r1, v1, tau1 = workloads.plummer(4096, rng=workloads.rng_for(1, 100))
    h.evolve(dev(m1), dev(r1), dev(v1), tau1, PLUMMER_HARVEST_STEPS)
    after_plummer = min(h.harvest_end(), cap - 1)
    h.harvest_begin(rows[after_plummer:], GUESS_DOMAIN)
    m2, r2, v2, tau2 = workloads.cluster(rng=workloads.rng_for(2, 100))
    h.evolve(dev(m2), dev(r2), dev(v2), tau2, harvest_steps)
    offered = after_plummer + h.harvest_end()
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    nrows = min(offered, cap)
    progress(f"harvest done: {nrows} rows in {t_harvest:.1f} s")
    t0 = time.perf_counter()
    model, hist = h.mlp_fit(rows[:nrows], GUESS_DOMAIN, epochs=20, batch=4096, seed=1)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    progress(f"training done in {t_fit:.1f} s")
    del rows
    h.close()

    # Plain (no model: the plain kernel alone) and learned runs alternate,
    # each from the same initial state, so that clock and thermal drift over
    # the run weigh on both alike; the median of the repeats is reported.
    handles = {GUESS_ANALYTIC: Sakura(0), GUESS_LEARNED: Sakura(0, guess=GUESS_LEARNED)}
    handles[GUESS_LEARNED].set_guess_model(model)
    walls = {GUESS_ANALYTIC: [], GUESS_LEARNED: []}
    stats = {}
    for _ in range(LEARNED_REPEATS):
        for mode, hh in handles.items():
            mt, rt, vt = dev(m), dev(r), dev(v)
            if warmup:
                hh.evolve(mt, rt, vt, tau, warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = hh.evolve(mt, rt, vt, tau, steps, stats=True)
            torch.cuda.synchronize()
            walls[mode].append(time.perf_counter() - t0)
            stats[mode] = st
        progress("learned: one plain and one learned run done")
    hp, hl = handles[GUESS_ANALYTIC], handles[GUESS_LEARNED]
    st_l = stats[GUESS_LEARNED]
    # the evaluations the plain starter takes in the network's domain (an
    # untimed run of the plain starter with the model loaded for statistics)
    hd = Sakura(0, guess=GUESS_ANALYTIC)
    hd.set_guess_model(model)
    mt, rt, vt = dev(m), dev(r), dev(v)
    if warmup:
        hd.evolve(mt, rt, vt, tau, warmup)
    st_p = hd.evolve(mt, rt, vt, tau, steps, stats=True)
    hd.close()
    wall_p = float(np.median(walls[GUESS_ANALYTIC]))
    wall_l = float(np.median(walls[GUESS_LEARNED]))
    n = len(m)
    pairs = n * (n - 1) // 2
    value = pairs * steps / wall_l
    # final residuals of the Kepler equation: one step of each starter with the
    # diagnostic kernels (every solve evaluated once more at its root)
    resid = {}
    for name, guess in (("plain", GUESS_ANALYTIC), ("learned", GUESS_LEARNED)):
        hr = Sakura(0, guess=guess, histogram=True)
        hr.set_guess_model(model)
        _, _, sr = gpu_one_step(hr, torch, m, r, v, tau)
        hr.close()
        resid[name] = {"max_rel_residual_all_solves": sr["max_rel_residual"],
                       "domain_pairs": sr["guess_domain_pairs"],
                       "domain_mean_iters": sr["guess_domain_iters"] /
                       max(sr["guess_domain_pairs"], 1)}
    parity = None
    if oracle_step is not None:
        rg, vg, _ = gpu_one_step(hl, torch, m, r, v, tau)
        er, ev = step_error(rg, vg, oracle_step[0], oracle_step[1], r, v)
        parity = {"err_r": er, "err_v": ev, "rows": int(n), "tol": 1e-12}
    out = {
        "value": value, "unit": "pair-solves/s", "vs_plain": wall_p / wall_l,
        "plain_value_interleaved": pairs * steps / wall_p,
        "repeats": LEARNED_REPEATS,
        "ms_per_step": wall_l * 1e3 / steps,
        "pair_kernel_ms": st_l["pair_kernel_ms"] / max(st_l["pair_launches"], 1),
        "domain": GUESS_DOMAIN,
        "domain_pairs_per_step": st_l["guess_domain_pairs"] / steps,
        "domain_mean_iters_plain": st_p["guess_domain_iters"] / max(st_p["guess_domain_pairs"], 1),
        "domain_mean_iters_learned": st_l["guess_domain_iters"] / max(st_l["guess_domain_pairs"], 1),
        "max_iters_plain": st_p["iters_max"], "max_iters_learned": st_l["iters_max"],
        "mean_kepler_iters": st_l["iters_total"] / max(st_l["pair_solves"], 1),
        "network_starts": st_l["guess_learned"], "restarts": st_l["guess_restarts"],
        "final_residual": resid,
        "training": {"harvest": f"{PLUMMER_HARVEST_STEPS} steps of an independent N=4096 "
                                f"Plummer sphere and {harvest_steps} steps of an independent "
                                f"N=16384 cluster (seed offset 100), plain starter",
                     "rows": int(nrows), "harvest_s": t_harvest, "fit_s": t_fit,
                     "epochs": 20, "val_mse_scaled": hist[-1]},
        "err_vs_oracle": parity,
    }
    hp.close()
    # the batched ensemble with the same network (few of its pairs reach the domain)
    off, mb, rb, vb, taub = workloads.ensemble()
    sizes = np.diff(off)
    bp = int(np.sum(sizes * (sizes - 1) // 2))
    mt, rt, vt, dtt = dev(mb), dev(rb), dev(vb), dev(taub)
    hl.autotune_batch(off, mt, rt, vt, dtt, probe_steps=8)
    hl.batch_evolve(off, mt, rt, vt, dtt, 256)  # warm-up: the graph of the timed call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sb = hl.batch_evolve(off, mt, rt, vt, dtt, 256, stats=True)
    torch.cuda.synchronize()
    wb = time.perf_counter() - t0
    out["batched"] = {"value": bp * 256 / wb, "unit": "pair-solves/s",
                      "domain_pairs": sb["guess_domain_pairs"],
                      "domain_mean_iters": sb["guess_domain_iters"] / max(sb["guess_domain_pairs"], 1),
                      "network_starts": sb["guess_learned"]}
    hl.close()
    return out


def accuracy_study(torch):
    """The paper's accuracy studies on the GPU (synthetic inputs): the relative
    energy error after one N-body time unit of the 128-star Plummer sphere
    around a black hole of q star masses, for tau = 1e-3, 1e-4, 1e-5 (Sec. 3.2),
    and after one outer period of two circular binaries on a circular outer
    orbit with a_out/a_in = 10, 100, 1000 (Sec. 3.1)."""
    from paper_1402_3325_amd import workloads
    from paper_1402_3325_amd.sakura import Sakura
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    h = Sakura(0)
    t0 = time.perf_counter()

    def rel_de(m, r, v, tau, nsteps):
        mt, rt, vt = dev(m), dev(r), dev(v)
        e0 = h.energy(mt, rt, vt)["E"]
        h.evolve(mt, rt, vt, tau, nsteps)
        e1 = h.energy(mt, rt, vt)["E"]
        return abs((e1 - e0) / e0)

    pbh = {}
    for q in (1.0, 1e1, 1e2, 1e3, 1e6, 1e9, 1e12):
        m, r, v = workloads.plummer_bh(q=q)
        pbh[f"{q:.0e}"] = {f"{tau:.0e}": rel_de(m, r, v, tau, int(round(1.0 / tau)))
                           for tau in (1e-3, 1e-4, 1e-5)}
    h4 = {}
    for ratio in (10.0, 100.0, 1000.0):
        m, r, v, P = workloads.hierarchical4(ratio)
        h4[f"{ratio:.0f}"] = {f"{tau:.0e}": rel_de(m, r, v, tau, int(round(P / tau)))
                              for tau in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5)}
    h.close()
    return {"study": "relative energy error |dE/E|, G = 1",
            "plummer_bh": {"workload": "128 equal-mass Plummer stars + central black hole of "
                                       "q star masses, virial, total mass 1; 1 time unit",
                           "dE_over_E": pbh},
            "hierarchical4": {"workload": "two circular binaries (masses 1/4, a_in = "
                                          "1/ratio) on a circular outer orbit a_out = 1; "
                                          "one outer period",
                              "dE_over_E": h4},
            "seconds": time.perf_counter() - t0}


SCHEME_NAMES = {0: "psi", 1: "unmerged", 2: "triple_jump"}
SCHEME_STAGES = {0: 1, 1: 2, 2: 3}


def schemes(lib, torch, m, r, v, tau, steps=32, warmup=8):
    """The compositions of the step (Sec. 2.2) on the GPU: throughput of each
    on the benchmark workload (every stage is one launch of the tile kernel),
    and the convergence order each reaches on a 64-star Plummer sphere over
    1/8 time unit (self-convergence against the triple jump with 16x smaller
    steps)."""
    from paper_1402_3325_amd import workloads
    n = len(m)
    pairs = n * (n - 1) // 2
    out = {}
    mt = torch.tensor(m, dtype=torch.float64, device="cuda")
    for sid, name in SCHEME_NAMES.items():
        rt = torch.tensor(r, dtype=torch.float64, device="cuda")
        vt = torch.tensor(v, dtype=torch.float64, device="cuda")
        lib.evolve_scheme(mt, rt, vt, tau, warmup, sid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = lib.evolve_scheme(mt, rt, vt, tau, steps, sid, stats=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"pair_solves_per_s": st["pair_solves"] / wall,
                     "ms_per_step": wall * 1e3 / steps,
                     "pair_launches_per_step": st["pair_launches"] / steps,
                     "pair_kernel_ms": st["pair_kernel_ms"] / max(st["pair_launches"], 1),
                     "mean_kepler_iters": st["iters_total"] / max(st["pair_solves"], 1)}
    ms, rs, vs, _ = workloads.plummer(64, rng=np.random.default_rng(64))
    T = 0.125
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    def run(sid, nsteps):
        rt, vt = dev(rs), dev(vs)
        lib.evolve_scheme(dev(ms), rt, vt, T / nsteps, nsteps, sid)
        return rt.cpu().numpy()

    ref = run(2, 1024)
    rrms = float(np.sqrt(np.mean(np.sum(rs ** 2, axis=1))))
    conv = {}
    for sid, name in SCHEME_NAMES.items():
        errs = [float(np.max(np.abs(run(sid, k) - ref))) / rrms for k in (16, 32, 64)]
        conv[name] = {"steps": [16, 32, 64],
                      "pair_solves": [k * SCHEME_STAGES[sid] * 64 * 63 // 2 for k in (16, 32, 64)],
                      "err_r": errs,
                      "order": [float(np.log2(errs[i] / errs[i + 1])) for i in range(2)]}
    out["convergence"] = {"workload": "64-star Plummer sphere, T = 1/8, reference: triple jump "
                                      "with 1024 steps", "by_scheme": conv}
    return out


def hybrid(lib, torch, m, r, v, tau, steps, warmup, etas=(0.01, 0.03)):
    """The close-pair hybrid on the benchmark workload: Kepler solves only for
    pairs with tau sqrt(mu/r^3) > eta or tau |W|/r > eta, the eq. (28) kick
    for the rest.  Pair interactions per second (every pair is still
    interacted with each step), the Kepler pairs per step, and the accuracy
    against the all-Kepler step: the difference after one step from the same
    state (the kicks' local error), and over the same warm-up + timed steps the
    relative energy change of each run and their final-state difference (the
    latter dominated by the chaotic growth of small differences)."""
    n = len(m)
    pairs = n * (n - 1) // 2
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    mt = dev(m)
    e0 = lib.energy(mt, dev(r), dev(v))["E"]
    rk, vk = dev(r), dev(v)
    lib.evolve(mt, rk, vk, tau, warmup + steps)
    ek = lib.energy(mt, rk, vk)["E"]
    rrms = float(np.sqrt(np.mean(np.sum(r ** 2, axis=1))))
    vrms = float(np.sqrt(np.mean(np.sum(v ** 2, axis=1))))
    r1, v1 = dev(r), dev(v)
    lib.evolve(mt, r1, v1, tau, 1)  # one all-Kepler step: the hybrid's local error against it
    out = {"workload": "the benchmark workload, warm-up + timed steps from the same start",
           "kepler_all": {"dE_over_E": abs((ek - e0) / e0)}, "by_eta": {}}
    for eta in etas:
        rt, vt = dev(r), dev(v)
        lib.set_hybrid(eta)
        try:
            rs, vs = dev(r), dev(v)
            lib.evolve(mt, rs, vs, tau, 1)
            one = {"max_dr_over_rrms": float((rs - r1).abs().max()) / rrms,
                   "max_dv_over_vrms": float((vs - v1).abs().max()) / vrms}
            lib.evolve(mt, rt, vt, tau, warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = lib.evolve(mt, rt, vt, tau, steps, stats=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        finally:
            lib.set_hybrid(0.0)
        eh = lib.energy(mt, rt, vt)["E"]
        dr = float((rt - rk).abs().max()) / rrms
        out["by_eta"][str(eta)] = {
            "pair_interactions_per_s": pairs * steps / wall,
            "ms_per_step": wall * 1e3 / steps,
            "pair_kernel_ms": st["pair_kernel_ms"] / max(st["pair_launches"], 1),
            "kepler_pairs_per_step": st["pair_solves"] / steps,
            "kicked_pairs_per_step": st["pair_kicks"] / steps,
            "mean_kepler_iters": st["iters_total"] / max(st["pair_solves"], 1),
            "dE_over_E": abs((eh - e0) / e0),
            "max_dr_vs_kepler_all_over_rrms": dr,
            "one_step_vs_kepler_all": one}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m, r, v, tau, one_core_s=4.0):
    """The oracle (plain C, OpenMP over rows, ordered pairs as in Listing 1):
    one full step of the same workload on every host core it is given (its
    output is also the reference of the GPU step's error over every row), and
    a sample of rows of that step on one core.  Each pair is solved from both
    of its ends, as in Listing 1, so unordered pairs advance at half the
    ordered rate."""
    import oracle
    n = len(m)
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    ro, vo = oracle.step(m, r, v, tau)
    el = time.perf_counter() - t0
    ordered = n * (n - 1)
    # one core: rows spread over the step, sized to about one_core_s
    oracle.set_num_threads(1)
    try:
        probe = np.linspace(0, n - 1, 16).astype(np.int64)
        t1 = time.perf_counter()
        oracle.step_rows(m, r, v, tau, probe)
        per_row = (time.perf_counter() - t1) / len(probe)
        nrows = int(min(n, max(16, one_core_s / max(per_row, 1e-9))))
        rows = np.linspace(0, n - 1, nrows).astype(np.int64)
        t1 = time.perf_counter()
        oracle.step_rows(m, r, v, tau, rows)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(cores)
    one = nrows * (n - 1) / el1
    out = {"value": ordered / el / 2.0, "unit": "pair-solves/s", "cores": cores,
           "kind": "oracle",
           "sample": f"one full step of the same workload (all {n} rows, {ordered} ordered "
                     f"pair solves: each of the {ordered // 2} pairs solved from both ends as "
                     f"in Listing 1) in {el:.2f} s; value counts unordered pairs",
           "ordered_solves_per_s": ordered / el,
           "one_core": {"ordered_solves_per_s": one, "pair_solves_per_s": one / 2.0,
                        "sample": f"{nrows} rows of the same step, {el1:.2f} s"},
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    return out, (ro, vo)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the warm-up lets the clocks settle (the pair kernel's launches speed up
    # over the first ~30 ms of load)
    ap.add_argument("--steps", type=int, default=256)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-schemes", action="store_true")
    ap.add_argument("--no-hybrid", action="store_true")
    # about 1e7 rows: the cluster yields ~350 rows per step in the domain
    ap.add_argument("--harvest-steps", type=int, default=30000)
    ap.add_argument("--clock-settle-ms", type=float, default=400.0,
                    help="untimed steps before the warm-up, run until this long has passed "
                         "(the pair kernel's launches speed up over the first ~30 ms of load "
                         "while the clocks rise)")
    ap.add_argument("--accuracy", action="store_true",
                    help="only run the accuracy studies (energy error vs mass ratio and "
                         "binary hierarchy) and print their JSON line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (x4), to scale "
                         "the rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy, "launches": 4}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus N > 1 is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1402_3325_amd import workloads
    from paper_1402_3325_amd.sakura import Sakura

    if args.accuracy:
        print(json.dumps(accuracy_study(torch)), flush=True)
        return

    m, r, v, tau, _ = workloads.config(2)
    n = len(m)
    pairs = n * (n - 1) // 2
    lib = Sakura(0)

    mt, rt, vt = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (m, r, v))
    # untimed: bring the clocks to their steady level on a copy of the state
    settle_steps = 0
    if args.clock_settle_ms > 0:
        rs, vs = rt.clone(), vt.clone()
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < args.clock_settle_ms:
            lib.evolve(mt, rs, vs, tau, 16)
            settle_steps += 16
        del rs, vs
    if args.warmup:
        lib.evolve(mt, rt, vt, tau, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = lib.evolve(mt, rt, vt, tau, args.steps, stats=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"timed block done: {wall * 1e3 / args.steps:.3f} ms per step")

    k_mean = st["iters_total"] / max(st["pair_solves"], 1)
    pair_ms = st["pair_kernel_ms"] / max(st["pair_launches"], 1)
    fl = flops_per_pair(k_mean) * pairs
    achieved = fl / (pair_ms * 1e-3) / 1e12
    prof = measured_profile()
    traffic = prof["bytes_per_launch"] if prof else None


    out = {
        "metric": METRIC,
        "value": pairs * args.steps / wall,
        "unit": "pair-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cluster: 16383 Plummer stars (10% in binaries) + central "
                               "mass 0.01, N=16384, tau=1/2048",
                   "n": n, "pairs_per_step": pairs, "guess": "analytic"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic},
        "flops_per_pair": flops_per_pair(k_mean),
        "flops_model": f"{FLOPS_SETUP} + {FLOPS_PER_ITER} k, k = mean Kepler evaluations "
                       "per solve",
        # the same launch against the work the kernel's source does per pair,
        # and (from the committed counters, null once the kernel sources
        # change) against the FP64 work the hardware counted, at 2.4 GHz and
        # at the clock measured during the kernel
        "roofline_kernel_count": {
            "flops_per_pair": kernel_flops_per_pair(k_mean),
            "frac": kernel_flops_per_pair(k_mean) * pairs / (pair_ms * 1e-3) / 1e12 /
            PEAK_FP64_TFLOPS},
        "roofline_hardware_counters": ({
            "hw_fp64_flops_per_pair": prof["hw_fp64_flops_per_pair"],
            "frac": prof["hw_fp64_flops_per_pair"] * pairs / (pair_ms * 1e-3) / 1e12 /
            PEAK_FP64_TFLOPS,
            "clock_ghz": prof["clock_ghz"],
            "frac_at_measured_clock": prof["hw_fp64_flops_per_pair"] * pairs /
            (pair_ms * 1e-3) / 1e12 / (PEAK_FP64_TFLOPS * prof["clock_ghz"] / 2.4),
            "valu_busy": prof["valu_busy"],
            "profiled_launch_ms": prof.get("launch_ms")} if prof else None),
        "pair_kernel_ms": pair_ms,
        "call_ms_events": st["call_ms"],
        "clock_settle": {"steps": settle_steps, "ms": args.clock_settle_ms},
        "mean_kepler_iters": k_mean,
        "max_kepler_iters": st["iters_max"],
        "fallbacks": st["fallbacks"],
        "kernel_source_hash": kernel_source_hash(),
        "err_vs_oracle": None,
    }
    if not args.no_schemes:
        out["schemes"] = schemes(lib, torch, m, r, v, tau)
        progress("schemes done")
    if not args.no_parity:
        out["plummer4096"] = plummer4096(lib, torch)
        progress("N = 4096 Plummer sphere done")
    if not args.no_hybrid:
        out["hybrid"] = hybrid(lib, torch, m, r, v, tau, args.steps, args.warmup)
        progress("hybrid done")
    if not args.no_batched:
        out["batched"] = batched(lib, torch)
        progress("batched ensemble done")
    # the oracle's full step (the CPU baseline) is the reference of the GPU
    # step's error over every row, for the plain and the learned starter
    cpu = None
    oracle_step = None
    if not args.no_cpu_baseline:
        cpu, oracle_step = cpu_baseline(m, r, v, tau)
        progress("cpu baseline done")
    elif not args.no_parity:
        import oracle
        oracle_step = oracle.step(m, r, v, tau)
    if not args.no_parity:
        rg, vg, _ = gpu_one_step(lib, torch, m, r, v, tau)
        er, ev = step_error(rg, vg, oracle_step[0], oracle_step[1], r, v)
        out["err_vs_oracle"] = {"err_r": er, "err_v": ev, "rows": int(n), "tol": 1e-12}
    if not args.no_learned:
        out["learned"] = learned(torch, m, r, v, tau, args.steps, args.warmup,
                                 args.harvest_steps, oracle_step)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
