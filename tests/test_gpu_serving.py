"""Sweep serving on the GPU: continuous batching completes a small seeded
trace, classifies diverging requests, and gives each request the same
bits it gets when stepped alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_05197_amd as M
    M.lib()
    return M


def test_small_trace_served_and_classified(M):
    from paper_2110_05197_amd import serve
    trace = serve.make_trace(n=12, rate=200.0, seed=3, d2_sizes=(32, 48), d3_sizes=(16, 24),
                             steps_range=(100, 400))
    # one request that must diverge: Shan-Chen far beyond its stable range
    bad = trace[0]
    bad.params = M.make_params(lattice=M.D3Q19, model=M.SC_MP, nx=16, ny=16, nz=16, G=-12.0,
                               tau_R=0.52, rho0_R=2.0, rho0_B=0.2, precision=M.FP32)
    bad.case = "droplet"
    server = serve.Server(k_steps=25)
    done, wall = server.run(trace)
    assert len(done) == 12
    by = {r.rid: r for r in done}
    assert by[bad.rid].outcome == "diverged"
    for r in done:
        if r.outcome == "done":
            assert r.steps_done == r.steps
    s = serve.summarize(done, wall)
    print(s, flush=True)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_served_accuracy_against_fp64(M):
    """Every request of a small trace that finishes both ways ends close to
    its one-at-a-time FP64 solve after 200-600 steps.  Served at the default
    precision (FP32 below density ratio 100, FP64 from 100): FP64 requests
    bit for bit (the same per-node arithmetic, batched or alone), FP32 ones
    within 1e-4 relative max norm of rho_R, rho_B (measured up to 3e-5).
    Served FP32/mixed (mixed from 100): mixed requests within 1e-3, where the
    heavy colour's FP32 deviations carry the light phase's density to a few
    1e-4, as in the density-ratio-1000 parity case (measured up to 3.3e-4)."""
    from paper_2110_05197_amd import serve
    kw = dict(n=14, rate=500.0, seed=11, d2_sizes=(32, 48, 64), d3_sizes=(16, 24, 32), steps_range=(200, 600))
    ref, _ = serve.serve_one_at_a_time(serve.make_trace(**kw), keep_fields=True)
    for rule in ("gamma", "fp64"):
        done, _ = serve.Server(k_steps=50, keep_fields=True).run(serve.make_trace(precision_rule=rule, **kw))
        serve.compare_runs(done, ref, release_reference=False)
        acc = serve.accuracy(done)
        for r in sorted(done, key=lambda r: r.rid):
            print(rule, r.rid, r.params["model"], r.params["precision"], round(r.gamma, 1), r.outcome,
                  r.info.get("rho_err"), flush=True)
        print(rule, acc, flush=True)
        assert acc["all"]["requests"] >= 8
        assert acc["fp32"]["requests"] >= 2 and acc["fp32"]["rho_err"]["max"] <= 1e-4
        if rule == "gamma":
            assert acc["mixed"]["requests"] >= 2 and acc["mixed"]["rho_err"]["max"] <= 1e-3
        else:
            assert acc["fp64"]["requests"] >= 2 and acc["fp64"]["rho_err"]["max"] == 0.0


def test_served_result_equals_solo(M):
    """A request's final populations are the same bits served in a mix as
    stepped alone through the batch API."""
    from paper_2110_05197_amd import serve
    trace = serve.make_trace(n=5, rate=1000.0, seed=4, d2_sizes=(32,), d3_sizes=(16,),
                             steps_range=(150, 250))
    sims, results = [], []
    for r in trace:
        s = M.Sim(r.params)
        s.init_equilibrium(*serve.initial_fields(r))
        sims.append(s)
    b = M.Batch(sims, [r.steps for r in trace])
    for _ in range(30):
        b.step(10)
    st, steps = b.status()
    b.close()
    mixed = [s.export_f().cpu().numpy() for s in sims]
    for r, fm, stt in zip(trace, mixed, st):
        s = M.Sim(r.params)
        s.init_equilibrium(*serve.initial_fields(r))
        b1 = M.Batch([s], [r.steps])
        for _ in range(30):
            b1.step(10)
        st1, _ = b1.status()
        b1.close()
        assert st1[0] == stt
        assert np.array_equal(s.export_f().cpu().numpy(), fm)


def test_laplace_sweep_machinery(M):
    """The static-droplet sweep (sweeps.run) on a reduced case: R = 8, 12,
    density ratios 1 and 1000 in one batch (FP32 and FP64 groups), 60000
    steps: no divergence, the equimolar radius within 1 of the set one and
    the interface radius beyond it at density ratio 1000, sigma_cal within
    10 % of sigma_th at density ratio 1 (20 % at 1000, which equilibrates
    more slowly), and the Laplace error smaller at the larger radius at
    density ratio 1."""
    from paper_2110_05197_amd import sweeps
    orig = sweeps.cases
    try:
        sweeps.cases = lambda study, radii=(8, 12): [(R, g, 1.0) for g in (1, 1000) for R in radii]
        out = sweeps.run("density", steps=60000, radii=(8, 12), chunk=1000, log=lambda *a: None)
    finally:
        sweeps.cases = orig
    res = out["results"]
    assert len(res) == 4 and not any(m["diverged"] for m in res)
    for m in res:
        assert abs(m["sigma_cal"] - 0.01) < (0.001 if m["gamma"] == 1 else 0.002), m
        assert abs(m["R_equimolar"] - m["R0"]) < 1.0, m
        if m["gamma"] == 1000:
            assert m["R"] > m["R0"] + 2.0, m
    e = {m["R0"]: m["E"] for m in res if m["gamma"] == 1}
    assert e[12] < e[8], e


def test_laplace_sweep_served(M, orc):
    """The Laplace study's droplets as requests of the sweep server: the same
    results, bit for bit, as the batched sweep (R = 8, 12 at density ratios 1
    in FP32 and 100 in FP64, 64^3, 1000 steps), and one served FP64 member
    (R = 12, density ratio 100) element by element against the oracle's
    1000 steps of the same droplet (relative max norm of rho_R, rho_B within
    1e-10)."""
    from paper_2110_05197_amd import serve, sweeps
    orig = sweeps.cases
    try:
        sweeps.cases = lambda study, radii=(8, 12): [(R, g, 1.0) for g in (1, 100) for R in radii]
        a = sweeps.run("density", steps=1000, radii=(8, 12), chunk=250, log=lambda *x: None)
        b = sweeps.run("density", steps=1000, radii=(8, 12), chunk=250, log=lambda *x: None, via_server=True)
    finally:
        sweeps.cases = orig
    assert len(a["results"]) == len(b["results"]) == 4
    for ma, mb in zip(a["results"], b["results"]):
        for k in ("sigma_cal", "R", "R_equimolar", "E", "ekin_per_area", "steps", "diverged"):
            assert ma[k] == mb[k], (k, ma, mb)
    # one member against the oracle
    p = sweeps.case_params(M, 12, 100, 1.0)
    assert p["precision"] == M.FP64
    L = p["nx"]
    reqs = [serve.Request(0, 0.0, p, "droplet", 1000, 100.0, 1.0, sweeps.SIGMA, radius=12.0),
            serve.Request(1, 0.0, sweeps.case_params(M, 8, 1, 1.0), "droplet", 700, 1.0, 1.0, sweeps.SIGMA,
                          radius=8.0)]
    done, _ = serve.Server(k_steps=100, keep_fields=True, policy="shared").run(reqs)
    served = {r.rid: r for r in done}[0]
    assert served.outcome == "done" and served.steps_done == 1000
    rR, rB = serve.initial_fields(reqs[0])
    fo = orc.run(p, orc.init_equilibrium(p, rR, rB, None), 1000)
    ro_R, ro_B, _ = orc.moments(p, fo)
    g = tuple(t.cpu().numpy() for t in served.final)
    err = serve.density_error(g, (ro_R, ro_B))
    print("served FP64 member against the oracle:", err, flush=True)
    assert err <= 1e-10


def test_ekin_sweep_machinery(M):
    """The CG-vs-SC stationary-droplet study (sweeps.run_ekin) on a reduced
    case, R = 20 in 64^3, 4000 steps: SC at two couplings, CG at two sigmas
    for density ratios 1 and 1000, one batch of three groups.  No
    divergence; SC droplets keep densities near the flat coexistence pair of
    their coupling, with a larger density ratio and a larger positive sigma
    at the stronger coupling; CG spurious-current energy grows with sigma;
    the batch run in four recorded segments keeps each droplet's E_kin
    history, whose last entry is the final value."""
    from paper_2110_05197_amd import serve, sweeps
    out = sweeps.run_ekin(steps=4000, chunk=500, sigmas=(0.01, 0.1), gammas=(1, 1000), couplings=(-4.8, -5.6),
                          record_every=1000, log=lambda *a: None)
    sc, cg = out["sc"], out["cg"]
    assert len(sc) == 2 and len(cg) == 4
    assert not any(m["diverged"] for m in sc + cg)
    for m in sc:
        liq, gas = serve.sc_coexistence(m["G"])
        assert abs(m["rho_in"] - liq) / liq < 0.1, m
        assert 0.5 * gas < m["rho_out"] < 2.0 * gas, m
        assert abs(m["R"] - sweeps.EKIN_R) < 2.0, m
        assert m["sigma"] > 0, m
    weak, strong = sc
    assert strong["ratio"] > weak["ratio"] and strong["sigma"] > weak["sigma"]
    for g in (1, 1000):
        e = {m["sigma"]: m["ekin"] for m in cg if m["gamma"] == g}
        assert e[0.1] > e[0.01] > 0, (g, e)
    assert set(out["fits"]) == {"SC", "CG gamma=1", "CG gamma=1000"}
    for m in cg:      # recorded in four segments of 1000 steps; the last equals the final E_kin
        assert [h[0] for h in m["ekin_history"]] == [1000, 2000, 3000, 4000] and m["steps"] == 4000
        assert m["ekin_history"][-1][1] == m["ekin"]
        assert m["settle_step"] in (1000, 2000, 3000, 4000)


def test_shortest_work_first_admission(M):
    """Policy "swf": with every request arrived and a node budget that holds
    only a few lattices, requests are admitted in order of the work they
    need, and all of them finish with the same outcome as under "shared"."""
    from paper_2110_05197_amd import serve
    kw = dict(n=10, rate=1e6, seed=5, d2_sizes=(32, 48, 64), d3_sizes=(16, 32), steps_range=(100, 600))
    trace = serve.make_trace(**kw)
    need = {r.rid: serve.work(r) for r in trace}
    done, _ = serve.Server(k_steps=25, policy="swf", max_nodes=3 * 32 * 32 * 32).run(trace)
    assert len(done) == 10
    by = sorted(done, key=lambda r: need[r.rid])
    for a, b in zip(by, by[1:]):
        if need[a.rid] < need[b.rid]:
            assert a.admitted <= b.admitted, (a.rid, b.rid)
    shared, _ = serve.Server(k_steps=25, policy="shared").run(serve.make_trace(**kw))
    assert {r.rid: r.outcome for r in done} == {r.rid: r.outcome for r in shared}


def test_served_one_pass_equals_solo(M):
    """Requests on 64^3 boxes run the batched one-pass kernel when served;
    their populations equal a solo run's, bit for bit."""
    from paper_2110_05197_amd import serve
    trace = serve.make_trace(n=4, rate=1e6, seed=6, d2_sizes=(32,), d3_sizes=(64,), steps_range=(60, 120))
    for r in trace:   # colour-gradient requests of the trace's gamma and sigma, FP32, 64^3
        p = M.make_params(lattice=M.D3Q19, model=M.CG, nx=64, ny=64, nz=64, precision=M.FP32,
                          rho0_R=r.gamma, rho0_B=1.0, tau_R=0.8, tau_B=0.6)
        r.params = M.params_from_sigma(p, r.sigma)
    sims = []
    for r in trace:
        s = M.Sim(r.params)
        s.init_equilibrium(*serve.initial_fields(r))
        sims.append(s)
    b = M.Batch(sims, [r.steps for r in trace])
    assert b.kernels() == [M.KERNEL_FUSED] * 4
    for _ in range(13):
        b.step(10)
    st, steps = b.status()
    b.close()
    assert st == [M.DONE] * 4
    for r, s, n in zip(trace, sims, steps):
        alone = M.Sim(dict(r.params, kernel=M.KERNEL_TWO_PASS))
        alone.init_equilibrium(*serve.initial_fields(r))
        st1, done1 = alone.step(int(n), check_every=int(n))
        assert done1 == n
        assert np.array_equal(alone.export_f().cpu().numpy(), s.export_f().cpu().numpy())
        alone.close()
        s.close()
