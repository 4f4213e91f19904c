"""Continuous-batching sweep serving over the mclbm batch API.

Requests are independent simulations (colour gradient or Shan-Chen, D2Q9 or
D3Q19, droplet or ligament, a density ratio, viscosity ratio and surface
tension) that arrive over time, as the parameter sweeps of the paper's
Laplace, stability and dynamics studies do.  The server keeps every admitted
simulation resident in HBM, admits arrivals as soon as memory allows, and
advances all resident simulations together: one batched launch per kernel
per group of equal (lattice, model, precision), captured as a HIP graph of K
steps and replayed.  Between replays it polls the per-simulation status
words, retires simulations that are done or diverged (NaN, Inf or rho <= 0)
and admits waiting ones.

The reference point is the same trace served one at a time in arrival order,
in FP64, with one simulation's two-pass kernels per launch and no graphs.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the trace starts
    params: dict            # mclbm_params fields
    case: str               # "droplet" or "ligament"
    steps: int
    gamma: float
    nu_ratio: float
    sigma: float
    radius: float = None    # droplet radius (default L/4)
    # filled in by the server
    admitted: float = math.nan
    finished: float = math.nan
    outcome: str = ""
    steps_done: int = 0
    info: dict = field(default_factory=dict)
    final: tuple = None     # (rho_R, rho_B) device FP64 tensors at the end, when kept
    obs: dict = None        # observables at the end, when kept


def sc_coexistence(G: float):
    """Liquid and gas densities (l, g) of the Shan-Chen multiphase model with
    psi = 1 - exp(-rho) under Guo forcing: p(l) = p(g) = p0 and the integral of
    (p0 - p) psi'/psi over [g, l] vanishes, with p = rho/3 + G psi^2 / 6.
    (nan, nan) at or above the critical coupling G = -4.

    The equation of state falls between its two spinodals, where dp/drho = 0,
    i.e. 1 + G x (1 - x) = 0 with x = exp(-rho).  For a pressure p0 between
    the local minimum and maximum, the gas root lies below the first spinodal
    and the liquid root above the second; the equal-area integral changes sign
    across that pressure range and is solved by bracketed root finding."""
    if not G < -4.0:
        return float("nan"), float("nan")
    from scipy.integrate import quad
    from scipy.optimize import brentq

    def psi(r):
        return -np.expm1(-r)

    def pr(r):
        return r / 3.0 + G * psi(r) ** 2 / 6.0

    disc = math.sqrt(1.0 + 4.0 / G)
    r_a = -math.log((1.0 + disc) / 2.0)     # local maximum of p
    r_b = -math.log((1.0 - disc) / 2.0)     # local minimum of p
    p_hi, p_lo = pr(r_a), max(pr(r_b), 0.0)

    def roots(p0):
        g = brentq(lambda r: pr(r) - p0, 0.0, r_a)
        hi = r_b + 1.0
        while pr(hi) < p0:
            hi *= 2.0
        l = brentq(lambda r: pr(r) - p0, r_b, hi)
        return l, g

    def area(p0):
        l, g = roots(p0)
        return quad(lambda r: (p0 - pr(r)) * math.exp(-r) / psi(r), g, l, limit=200)[0]

    span = p_hi - p_lo
    a, b = p_lo + 1e-12 * span, p_hi - 1e-12 * span
    if area(a) * area(b) > 0:
        return float("nan"), float("nan")
    p0 = brentq(area, a, b, xtol=1e-14 * max(1.0, abs(p_hi)))
    return roots(p0)


def sc_coexistence_ratio(G: float) -> float:
    """Liquid/gas density ratio of the Shan-Chen multiphase coexistence at G
    (nan at or above the critical coupling)."""
    l, g = sc_coexistence(G)
    return float(l / g)


_SC_TABLE = None


def sc_coupling_for_ratio(gamma: float) -> float:
    """G whose Shan-Chen coexistence has liquid/gas ratio gamma, interpolated
    in log(ratio) on a table of the coexistence solution over G in [-4.02, -6.5];
    ratios beyond the table clamp to its strongest coupling."""
    global _SC_TABLE
    if _SC_TABLE is None:
        Gs = np.linspace(-4.02, -6.5, 64)
        rs = np.array([sc_coexistence_ratio(g) for g in Gs])
        ok = np.isfinite(rs) & (rs > 1)
        Gs, rs = Gs[ok], rs[ok]
        order = np.argsort(rs)
        _SC_TABLE = (np.log(rs[order]), Gs[order])
    lr, Gs = _SC_TABLE
    target = math.log(gamma)
    G = float(np.interp(target, lr, Gs))
    if not lr[0] < target < lr[-1]:
        return G
    # two secant steps on log(ratio) from the table's bracketing entries
    k = int(np.searchsorted(lr, target))
    G0, f0 = float(Gs[k - 1]), float(lr[k - 1]) - target
    for _ in range(2):
        f1 = math.log(sc_coexistence_ratio(G)) - target
        if f1 == f0 or not math.isfinite(f1):
            break
        G, G0, f0 = G - f1 * (G - G0) / (f1 - f0), G, f1
    return G


def make_trace(n=256, rate=20.0, seed=0, d2_sizes=(64, 96, 128, 192, 256, 384, 512),
               d3_sizes=(64, 80, 96, 112, 128, 144, 160), steps_range=(1000, 20000),
               precisions=(1, 2), precision_rule="fp64", conserve_mass=False):
    """Seeded request trace: Poisson arrivals at `rate` per second; model CG
    or SC (p = 1/2); droplet (R = L/4) or ligament (R = L/8, aspect 5, capped
    to 0.8 L); D2Q9 or D3Q19 (p = 1/2) with L from the size lists; density
    ratio 10^U(0,3), viscosity ratio 10^U(0,2), sigma 10^U(-3,-1); steps
    U{steps_range}.  Storage precision, precision_rule "fp64": FP32 below
    density ratio 100 and FP64 from 100 on (FP32 and mixed storage carry the
    heavy colour's rounding into the light phase at high density ratios: its
    density and the spurious currents drift away from the FP64 solution over
    thousands of steps); "gamma": FP32 below 100 and mixed from 100 on;
    "random": drawn from `precisions`.  The draw is made under every rule,
    so the traces differ in precision only.  conserve_mass: the FP32 and
    mixed colour-gradient requests keep each colour's node mass to one
    rounding per step (mclbm_params.conserve_mass), which brings their
    densities closer to the FP64 solves at a few per cent of the step."""
    import paper_2110_05197_amd as M
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        model = "CG" if rng.random() < 0.5 else "SC"
        case = "droplet" if rng.random() < 0.5 else "ligament"
        d3 = rng.random() < 0.5
        L = int(rng.choice(d3_sizes if d3 else d2_sizes))
        gamma = 10 ** rng.uniform(0, 3)
        nu_ratio = 10 ** rng.uniform(0, 2)
        sigma = 10 ** rng.uniform(-3, -1)
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        prec = int(rng.choice(precisions))
        if precision_rule == "fp64":
            prec = M.FP64 if gamma >= 100.0 else M.FP32
        elif precision_rule == "gamma":
            prec = M.MIXED if gamma >= 100.0 else M.FP32
        elif precision_rule != "random":
            raise ValueError(f"unknown precision rule {precision_rule!r}")
        lattice = M.D3Q19 if d3 else M.D2Q9
        base = dict(lattice=lattice, nx=L, ny=L, nz=L if d3 else 1, precision=prec)
        # heavy fluid more viscous: nu_R = nu0 sqrt(r), nu_B = nu0 / sqrt(r)
        nu0 = 1.0 / 6.0
        nuR, nuB = nu0 * math.sqrt(nu_ratio), nu0 / math.sqrt(nu_ratio)
        if model == "CG":
            p = M.make_params(model=M.CG, rho0_R=gamma, rho0_B=1.0, tau_R=0.5 + 3 * nuR,
                              tau_B=0.5 + 3 * nuB,
                              conserve_mass=int(conserve_mass and prec in (M.FP32, M.MIXED)), **base)
            p = M.params_from_sigma(p, sigma)
        else:
            G = sc_coupling_for_ratio(gamma) if gamma > 1.5 else -4.5
            p = M.make_params(model=M.SC_MP, G=G, tau_R=1.0, rho0_R=2.0, rho0_B=0.2, **base)
        out.append(Request(rid, t, p, case, steps, gamma, nu_ratio, sigma))
    return out


def initial_fields(req: Request):
    """Droplet or ligament fields for a request (inputs recipe)."""
    p = req.params
    shape = (p["nz"], p["ny"], p["nx"])
    L = p["nx"]
    if p["model"] == 1:
        # SC multiphase: liquid droplet in vapour at the coexistence densities of G
        rhoL, rhoG = sc_coexistence(p["G"])
    else:
        rhoL, rhoG = p["rho0_R"], p["rho0_B"]
    if req.case == "droplet":
        rR, rB = inputs.droplet(shape, req.radius if req.radius else L / 4.0, rhoL, rhoG)
    else:
        R = L / 8.0
        rR, rB = inputs.ligament(shape, R, min(10 * R, 0.8 * L), rhoL, rhoG, axis=0)
    if p["model"] == 1:
        return rR + rB, None
    return rR, rB


def footprint(req: Request) -> int:
    import paper_2110_05197_amd as M
    return M.state_bytes(req.params)


def work(req: Request) -> int:
    """Lattice updates a request still needs."""
    p = req.params
    return (req.steps - req.steps_done) * p["nx"] * p["ny"] * p["nz"]


class Server:
    """Continuous batching: admit by free HBM, step resident sims together.

    policy "shared": every arrived request is admitted as soon as memory
    allows, and all resident simulations share the GPU.
    policy "swf" (shortest work first): arrived requests are admitted in
    order of the lattice updates they need, while the resident lattices hold
    at most `max_nodes` nodes; a request larger than that runs when nothing
    else is resident, and a request that arrives meanwhile waits for the next
    completion instead of slowing the running ones down.  No running
    simulation is preempted.  As with any shortest-first order, a long
    request waits while shorter ones keep arriving; on a finite trace it runs
    once they are served.  The default budget, 4 M nodes (a 160^3 lattice),
    keeps the GPU busy with the lattice sizes of the paper's sweeps while
    short requests finish early: on the 256-request trace the median latency
    fell from 41 s at 32 M nodes to 6.7 s at the same throughput.
    """

    def __init__(self, k_steps=100, use_graph=True, reserve_bytes=4 << 30, max_resident=512,
                 log=None, policy="swf", max_nodes=4 << 20, keep_fields=False):
        import torch
        if policy not in ("shared", "swf"):
            raise ValueError(f"unknown policy {policy!r}")
        self.k = k_steps
        self.use_graph = use_graph
        self.reserve = reserve_bytes
        self.max_resident = max_resident
        self.policy = policy
        self.max_nodes = max_nodes if policy == "swf" else None
        self.stream = torch.cuda.Stream()
        self.log = log or (lambda *a: None)
        self.keep_fields = keep_fields   # keep each finished request's final densities (on the device)

    def free_bytes(self):
        import torch
        free, total = torch.cuda.mem_get_info()
        return free

    def run(self, trace):
        import torch
        import paper_2110_05197_amd as M
        waiting = sorted(trace, key=lambda r: r.arrival)
        resident = []          # (req, sim, remaining)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        done = []
        nodes = lambda r: r.params["nx"] * r.params["ny"] * r.params["nz"]

        def candidates():
            """Arrived requests in admission order."""
            t = now()
            arrived = [r for r in waiting if r.arrival <= t]
            return sorted(arrived, key=work) if self.policy == "swf" else arrived

        def fits(req, resident_nodes):
            if len(resident) >= self.max_resident:
                return False
            if self.max_nodes is not None and resident and resident_nodes + nodes(req) > self.max_nodes:
                return False
            need = footprint(req) + 16 * nodes(req)
            return self.free_bytes() - need >= self.reserve or not resident

        with torch.cuda.stream(self.stream):
            while waiting or resident:
                # admit arrived requests while memory, slots and the node budget allow
                resident_nodes = sum(nodes(r) for (r, _, _) in resident)
                for req in candidates():
                    if not fits(req, resident_nodes):
                        break
                    waiting.remove(req)
                    sim = M.Sim(req.params, stream=self.stream)
                    rR, rB = initial_fields(req)
                    sim.init_equilibrium(rR, rB)
                    req.admitted = now()
                    resident.append([req, sim, req.steps])
                    resident_nodes += nodes(req)
                if not resident:
                    # idle until the next arrival
                    if waiting:
                        time.sleep(max(0.0, min(0.01, waiting[0].arrival - now())))
                    continue
                batch = M.Batch([s for (_, s, _) in resident], [r for (_, _, r) in resident],
                                stream=self.stream)
                # replay K-step graphs until somebody finishes or an arrival can be admitted
                while True:
                    batch.step(self.k, use_graph=self.use_graph)
                    st, steps = batch.status()
                    finished = [i for i, s in enumerate(st) if s != M.RUNNING]
                    cand = candidates()
                    admissible = bool(cand) and fits(cand[0], resident_nodes)
                    if finished or admissible:
                        break
                batch.close()
                keep = []
                for i, (req, sim, rem) in enumerate(resident):
                    rem_now = rem - steps[i]
                    req.steps_done += steps[i]
                    if st[i] == M.RUNNING:
                        keep.append([req, sim, rem_now])
                        continue
                    req.finished = now()
                    req.outcome = "done" if st[i] == M.DONE else "diverged"
                    if st[i] == M.DONE and sim.diverged():
                        req.outcome = "diverged"
                    if self.keep_fields and req.outcome == "done":
                        req.final = sim.moments()[:2]
                        req.obs = sim.observables()
                    done.append(req)
                    sim.close()
                    self.log(f"[serve] {req.rid} {req.outcome} after {req.steps_done} steps")
                resident = keep
        torch.cuda.synchronize()
        return done, now()


def density_error(a, ref):
    """Relative max-norm error of the densities a = (rho_R, rho_B) against
    ref: max over the components present of max|a_k - ref_k| / max|ref_k|."""
    err = 0.0
    for x, r in zip(a, ref):
        scale = float(np.abs(r).max())
        if scale > 0.0:
            err = max(err, float(np.abs(x - r).max()) / scale)
    return err


def serve_one_at_a_time(trace, check_every=1000, log=None, keep_fields=False):
    """Reference: FIFO, one simulation at a time, FP64, two-pass kernels, no
    graphs; a request cannot start before it arrives.  keep_fields: keep each
    finished request's final densities on the device (req.final)."""
    import torch
    import paper_2110_05197_amd as M
    log = log or (lambda *a: None)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    out = []
    for req in sorted(trace, key=lambda r: r.arrival):
        while now() < req.arrival:
            time.sleep(min(0.01, req.arrival - now()))
        p = dict(req.params, precision=M.FP64, kernel=M.KERNEL_TWO_PASS)
        sim = M.Sim(p)
        rR, rB = initial_fields(req)
        sim.init_equilibrium(rR, rB)
        req.admitted = now()
        st, done = sim.step(req.steps, check_every=check_every)
        torch.cuda.synchronize()
        req.steps_done = done
        req.finished = now()
        req.outcome = "diverged" if st == M.DIVERGED else "done"
        if keep_fields and req.outcome == "done":
            req.final = sim.moments()[:2]
            req.obs = sim.observables()
        sim.close()
        out.append(req)
        log(f"[fifo] {req.rid} {req.outcome}")
    return out, now()


def _rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else (0.0 if a == b else math.inf)


def compare_runs(served, reference, release_reference=True):
    """Per-request differences of `served` from `reference` (two runs of one
    trace that kept their final fields and observables), set in the served
    requests' info for those that finished on both sides:
      rho_err    relative max-norm error of rho_R, rho_B (density_error);
      volume_err relative difference of the red (liquid) volume;
      jump_err   relative difference of the density jump rho_in - rho_out
                 across the interface (the Laplace test's measure);
      ekin_ratio kinetic energy (spurious currents of a resting drop) over the
                 reference's.
    The served fields are released afterwards, and the reference's unless
    release_reference is false (to compare a second run against it)."""
    ref = {r.rid: r for r in reference}
    for r in served:
        q = ref.get(r.rid)
        if r.final is not None and q is not None and q.final is not None:
            a = tuple(t.cpu().numpy() for t in r.final)
            b = tuple(t.cpu().numpy() for t in q.final)
            r.info["rho_err"] = density_error(a, b)
            if r.obs is not None and q.obs is not None:
                o, p = r.obs, q.obs
                r.info["volume_err"] = _rel(o["red_volume"], p["red_volume"])
                r.info["jump_err"] = _rel(o["rho_in"] - o["rho_out"], p["rho_in"] - p["rho_out"])
                r.info["ekin_ratio"] = o["ekin"] / p["ekin"] if p["ekin"] > 0 else math.nan
                r.info["ekin"], r.info["ekin_ref"] = o["ekin"], p["ekin"]
    for r in list(served) + (list(reference) if release_reference else []):
        r.final = None


def _describe(r):
    return dict(rid=r.rid, model="CG" if r.params["model"] == 0 else "SC",
                lattice="D3Q19" if r.params["nz"] > 1 else "D2Q9", L=r.params["nx"],
                case=r.case, gamma=round(r.gamma, 2), nu_ratio=round(r.nu_ratio, 2),
                sigma=float(f"{r.sigma:.3g}"), steps=r.steps)


def accuracy(reqs):
    """Per storage precision (and over all): the number of compared requests,
    max and 99th percentile of rho_err, volume_err and jump_err, and the
    largest kinetic-energy ratio (see compare_runs), each maximum with the
    request it came from (worst)."""
    import paper_2110_05197_amd as M
    names = {M.FP32: "fp32", M.MIXED: "mixed", M.FP16: "fp16", M.FP64: "fp64"}
    out = {}
    groups = {"all": [r for r in reqs if "rho_err" in r.info]}
    for r in groups["all"]:
        groups.setdefault(names.get(r.params["precision"], "other"), []).append(r)
    for key, rs in groups.items():
        g = dict(requests=len(rs))
        worst = {}
        for name in ("rho_err", "volume_err", "jump_err"):
            fin = [r for r in rs if name in r.info and math.isfinite(r.info[name])]
            e = np.array([r.info[name] for r in fin])
            g[name] = dict(max=float(e.max()), p99=float(np.percentile(e, 99))) if len(e) else None
            if fin:
                worst[name] = _describe(max(fin, key=lambda r: r.info[name]))
        fin = [r for r in rs if math.isfinite(r.info.get("ekin_ratio", math.nan))]
        g["ekin_ratio_max"] = max(r.info["ekin_ratio"] for r in fin) if fin else None
        if fin:
            w = max(fin, key=lambda r: r.info["ekin_ratio"])
            worst["ekin_ratio"] = dict(_describe(w), ekin=w.info["ekin"], ekin_ref=w.info["ekin_ref"])
        g["worst"] = worst
        out[key] = g
    return out


def summarize(reqs, wall):
    lat = np.array([r.finished - r.arrival for r in reqs])
    lups = sum(r.steps_done * r.params["nx"] * r.params["ny"] * r.params["nz"] for r in reqs)
    outcomes = {}
    for r in reqs:
        key = f"{'CG' if r.params['model'] == 0 else 'SC'}:{r.outcome}"
        outcomes[key] = outcomes.get(key, 0) + 1
    div = [r for r in reqs if r.outcome == "diverged"]
    outcomes["diverged_gamma_min"] = round(min((r.gamma for r in div), default=float("nan")), 2)
    return dict(requests=len(reqs), wall_s=round(wall, 3),
                throughput_req_s=round(len(reqs) / wall, 4),
                glups=round(lups / wall / 1e9, 3),
                p50_latency_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_s=round(float(np.percentile(lat, 99)), 4),
                outcomes=outcomes)
