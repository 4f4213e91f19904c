"""Host logic of the sweep server: the Shan-Chen coexistence solver that maps a
requested density ratio to a coupling, the seeded trace and the summary
statistics.  No GPU."""
import math

import numpy as np
import pytest

from paper_2110_05197_amd import serve


def _pressure(G, r):
    return r / 3.0 + G * (1.0 - math.exp(-r)) ** 2 / 6.0


@pytest.mark.parametrize("G", [-4.05, -4.5, -5.0, -5.5, -6.0, -6.3])
def test_coexistence_equal_pressure_and_area(G):
    from scipy.integrate import quad
    l, g = serve.sc_coexistence(G)
    assert 0 < g < math.log(2.0) < l
    p0 = _pressure(G, l)
    assert abs(_pressure(G, g) - p0) < 1e-12
    area = quad(lambda r: (p0 - _pressure(G, r)) * math.exp(-r) / (1 - math.exp(-r)), g, l,
                limit=200)[0]
    assert abs(area) < 1e-10


def test_coexistence_matches_oracle_flat_interface(orc):
    """A flat liquid slab in the oracle at G = -5 relaxes (5000 steps) to the
    solver's coexistence densities."""
    from paper_2110_05197_amd import inputs
    G = -5.0
    shape = (1, 3, 64)
    p = orc.make_params(lattice=0, model=1, nx=64, ny=3, nz=1, G=G, tau_R=1.0, rho0_R=2.0,
                        rho0_B=0.15)
    rR, rB = inputs.slab(shape, 32.0, 2.0, 0.15, axis=0)
    f = orc.run(p, orc.init_equilibrium(p, rR + rB, None), 5000)
    rho, _, _ = orc.moments(p, f)
    l, g = serve.sc_coexistence(G)
    assert abs(rho[0, 1, 32] - l) / l < 1e-4
    assert abs(rho[0, 1, 0] - g) / g < 1e-4


def test_coexistence_monotone_and_critical_limit():
    Gs = np.linspace(-4.02, -6.3, 20)
    ratios = [serve.sc_coexistence_ratio(G) for G in Gs]
    assert all(b > a for a, b in zip(ratios, ratios[1:]))
    assert math.isnan(serve.sc_coexistence_ratio(-4.0))
    assert math.isnan(serve.sc_coexistence_ratio(-3.0))
    l, g = serve.sc_coexistence(-4.001)
    assert abs(l - math.log(2.0)) < 0.1 and abs(g - math.log(2.0)) < 0.1


@pytest.mark.parametrize("gamma", [2.0, 10.0, 100.0, 900.0])
def test_coupling_for_ratio_round_trip(gamma):
    G = serve.sc_coupling_for_ratio(gamma)
    assert abs(serve.sc_coexistence_ratio(G) - gamma) / gamma < 0.02


def test_trace_is_seeded():
    a = serve.make_trace(seed=3, n=20)
    b = serve.make_trace(seed=3, n=20)
    c = serve.make_trace(seed=4, n=20)
    key = lambda tr: [(r.arrival, r.params["nx"], r.params["model"], r.steps) for r in tr]
    assert key(a) == key(b) and key(a) != key(c)
    assert all(x.arrival < y.arrival for x, y in zip(a, a[1:]))


def test_trace_precision_rule():
    """Rule "fp64" (the default): FP64 storage exactly for density ratios >=
    100, FP32 below; rule "gamma": mixed storage there instead; the rest of
    the trace is the one the "random" rule draws."""
    import paper_2110_05197_amd as M
    d = serve.make_trace(seed=5, n=60)
    g = serve.make_trace(seed=5, n=60, precision_rule="gamma")
    r = serve.make_trace(seed=5, n=60, precision_rule="random")
    assert any(x.gamma >= 100 for x in d) and any(x.gamma < 100 for x in d)
    assert all(x.params["precision"] == (M.FP64 if x.gamma >= 100 else M.FP32) for x in d)
    assert all(x.params["precision"] == (M.MIXED if x.gamma >= 100 else M.FP32) for x in g)
    assert {x.params["precision"] for x in r} == {M.FP32, M.MIXED}
    strip = lambda d: {k: v for k, v in d.items() if k != "precision"}
    for t in (d, g):
        assert all(strip(a.params) == strip(b.params) and a.arrival == b.arrival
                   for a, b in zip(t, r))
    with pytest.raises(ValueError):
        serve.make_trace(seed=5, n=4, precision_rule="fp16")


def test_trace_conserve_mass_option():
    """conserve_mass=True marks exactly the FP32 and mixed colour-gradient
    requests (FP64 and Shan-Chen requests keep 0) and changes nothing else."""
    import paper_2110_05197_amd as M
    for rule in ("fp64", "gamma"):
        a = serve.make_trace(seed=6, n=60, precision_rule=rule)
        b = serve.make_trace(seed=6, n=60, precision_rule=rule, conserve_mass=True)
        assert all(x.params["conserve_mass"] == 0 for x in a)
        for x, y in zip(a, b):
            want = int(x.params["model"] == M.CG and x.params["precision"] in (M.FP32, M.MIXED))
            assert y.params["conserve_mass"] == want
            assert dict(y.params, conserve_mass=0) == x.params and y.arrival == x.arrival
        assert any(y.params["conserve_mass"] for y in b)


def test_initial_fields_sc_at_coexistence():
    tr = serve.make_trace(seed=0, n=40, d2_sizes=(64,), d3_sizes=(32,))
    sc = [r for r in tr if r.params["model"] == 1]
    assert sc
    for r in sc[:4]:
        rho, none = serve.initial_fields(r)
        assert none is None
        l, g = serve.sc_coexistence(r.params["G"])
        assert g * (1 - 1e-9) <= rho.min() < g * (1 + 1e-3)
        assert g + 0.8 * (l - g) < rho.max() <= l * (1 + 1e-9)


def test_summarize_percentiles():
    reqs = []
    for i in range(10):
        r = serve.Request(i, float(i), dict(model=0, nx=10, ny=10, nz=1), "droplet", 100, 1, 1, 0.01)
        r.finished = r.arrival + (i + 1)
        r.steps_done = 100
        r.outcome = "done"
        reqs.append(r)
    s = serve.summarize(reqs, 20.0)
    assert s["requests"] == 10 and s["throughput_req_s"] == 0.5
    assert s["p50_latency_s"] == pytest.approx(5.5) and s["p99_latency_s"] == pytest.approx(9.91)
    assert s["glups"] == pytest.approx(10 * 100 * 100 / 20 / 1e9, abs=1e-3)


def test_accuracy_summary_names_the_worst_requests():
    """accuracy(): counts, maxima and the request each maximum came from, per
    storage precision and over all; requests without a comparison are left
    out, a non-finite ratio does not become the maximum."""
    import paper_2110_05197_amd as M
    tr = serve.make_trace(seed=1, n=6, precision_rule="random")
    errs = [1e-5, 3e-4, 2e-5, 7e-6, 5e-5, None]
    for r, e in zip(tr, errs):
        r.params["precision"] = M.FP32 if r.rid % 2 == 0 else M.MIXED
        if e is not None:
            r.info.update(rho_err=e, volume_err=e / 10, jump_err=e / 100,
                          ekin_ratio=math.nan if r.rid == 1 else 1 + 10 * e,
                          ekin=1.0, ekin_ref=1.0)
    acc = serve.accuracy(tr)
    assert acc["all"]["requests"] == 5
    assert acc["all"]["rho_err"]["max"] == 3e-4 and acc["all"]["worst"]["rho_err"]["rid"] == 1
    assert acc["all"]["worst"]["ekin_ratio"]["rid"] == 4      # rid 1 has a nan ratio
    fp32 = [r for r in tr if r.params["precision"] == M.FP32 and "rho_err" in r.info]
    assert acc["fp32"]["requests"] == len(fp32)
    assert acc["fp32"]["rho_err"]["max"] == max(r.info["rho_err"] for r in fp32)
    assert acc["mixed"]["worst"]["volume_err"]["rid"] == 1
