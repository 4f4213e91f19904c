"""Parameter sweeps of the paper's static-droplet studies, run as one batch of
independent simulations on the GPU (the batch API of the library).

Study "density" (Laplace test, section 3.1): a 3-D colour-gradient droplet of
radius R = 8, 12, 16, 20 at density ratios rho_R/rho_B = 1, 10, 100, 1000 and
viscosity ratio 1; study "viscosity": density ratio 1 and viscosity ratios
nu_R/nu_B = 1, 2, 5, 10, 100.  sigma_th = 0.01 throughout (Eq. sigmaA).  After
the equilibration each droplet gives

* sigma_cal from Young-Laplace in 3-D, dP = 2 sigma / R (Eq. YoungLaplace),
  with p_k = rho_k (1 - alpha_k) / 2 (Eq. CGpressure) from the
  epsilon-masked inside/outside densities (Eqs. rhoin, rhoout) and R the
  radius of the colour interface rho^N = 0, from the red volume
  sum (1 + rho^N)/2 (reading: the paper does not say how it measures R; at a
  density ratio this interface lies well out on the light side of the
  equimolar radius of the red mass, 14.0 against 8.4 for R = 8 at density
  ratio 1000, and only the interface radius gives the paper's finding that
  the error falls as the density ratio grows);
* the error E = |sigma_th - sigma_cal| / sigma_th;
* the kinetic energy of the spurious currents per droplet area,
  E_kin / A_d with A_d = 4 pi R^2 at the set radius;

and each series is fitted against the set radii R = 8 ... 20 with E ∝ R^b and
E_kin / A_d ∝ R^b, the fits the paper tabulates (Tables densErrors,
viscErrors, radiusErrors).

Study "ekin" (the stationary-droplet comparison of CG and SC, section
3.1.2): droplets of R = 20 in the same 64^3 periodic box, 10^5 steps,

* Shan-Chen multiphase (psi = 1 - exp(-rho), FP64) over couplings G inside
  the stable range the paper reports (4.2 < |G| < 6.5), each droplet started
  at the flat-interface coexistence densities of its G; measured: rho_in and
  rho_out at the droplet centre and the box corner, their ratio, sigma from
  Young-Laplace with p = rho/3 + G psi^2/6 and the equimolar radius, and the
  total kinetic energy E_kin;
* colour gradient at sigma_th = 0.001 ... 0.3 for density ratios 1, 10,
  100, 1000 (tau = 1 for both colours; FP32, FP64 from density ratio 100),
  E_kin at the end and every 5000 steps, with the step from which it stays
  within 5 % of its final value;

and E_kin ∝ sigma^b fitted per series (the paper: b = 2 for CG at every
density ratio, b = 3.3 for SC, whose density ratio stays below about 50).
Study "ekin-tau": the CG droplets at density ratio 1 with tau_R = 0.55,
0.625, 0.75, 0.875, 1 and tau_B = 1 (the viscosity variant of the same
comparison).

Readings: rho_B = 1 and rho_R = gamma (as for the other density-ratio cases);
the viscosity ratio r is split as nu_R = nu0 sqrt(r), nu_B = nu0 / sqrt(r)
with nu0 = 1/6, so that every tau stays in [0.55, 5.5]; the box is periodic,
64^3 for every radius (the domain of the Laplace section), the droplet
centred; FP64 for density ratios >= 100, FP32 otherwise.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs

PRINTED_B = {
    "density": {1: -2.02, 10: -1.81, 100: -1.82, 1000: -1.90},
    "viscosity": {1: -2.02, 2: -1.48, 5: -1.37, 10: -1.34, 100: -1.29},
    "ekin": {1: -0.59, 10: -0.85, 100: -1.02, 1000: -1.14},
}
RADII = (8, 12, 16, 20)
SIGMA = 0.01


LAPLACE_BOX = 64


def box_for(R: int) -> int:
    """Periodic cube of the Laplace section: 64^3 whatever the radius."""
    return LAPLACE_BOX


def case_params(M, R, gamma, nu_ratio, heavy=None):
    """Laplace-study droplet; FP32 below density ratio 100, `heavy` (default
    FP64) from 100 on: there the pressure jump is about 1e-3 of either
    phase's pressure, so sigma_cal needs rho_in to about 1e-4, which FP32
    storage of the heavy phase does not hold over 10^5 steps."""
    L = box_for(R)
    nu0 = 1.0 / 6.0
    nuR, nuB = nu0 * math.sqrt(nu_ratio), nu0 / math.sqrt(nu_ratio)
    prec = (M.FP64 if heavy is None else heavy) if gamma >= 100 else M.FP32
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=L, ny=L, nz=L, rho0_R=float(gamma),
                      rho0_B=1.0, tau_R=0.5 + 3 * nuR, tau_B=0.5 + 3 * nuB)
    return M.params_from_sigma(p, SIGMA)


def cases(study: str, radii=RADII):
    if study == "density":
        return [(R, g, 1.0) for g in (1, 10, 100, 1000) for R in radii]
    if study == "viscosity":
        return [(R, 1, r) for r in (1, 2, 5, 10, 100) for R in radii]
    raise ValueError(study)


def measure(obs, p, R0=None):
    """sigma_cal, E and E_kin / A_d of one equilibrated droplet (A_d at the
    set radius R0 when given, else at the interface radius)."""
    aR = 1.0 - (1.0 - p["alpha_B"]) * p["rho0_B"] / p["rho0_R"]   # Eq. gamma
    cR2, cB2 = (1.0 - aR) / 2.0, (1.0 - p["alpha_B"]) / 2.0
    R = (3.0 * obs["red_volume"] / (4.0 * math.pi)) ** (1.0 / 3.0)
    R_eq = (3.0 * obs["mass_R"] / (4.0 * math.pi * obs["rho_in"])) ** (1.0 / 3.0)
    dP = obs["rho_in"] * cR2 - obs["rho_out"] * cB2
    sigma_cal = dP * R / 2.0
    Ra = R if R0 is None else R0
    return dict(R=R, R_equimolar=R_eq, sigma_cal=sigma_cal, E=abs(SIGMA - sigma_cal) / SIGMA,
                ekin_per_area=obs["ekin"] / (4.0 * math.pi * Ra * Ra), eps=obs["eps_used"])


def fit_slope(R, y):
    R, y = np.asarray(R, float), np.asarray(y, float)
    ok = y > 0
    if ok.sum() < 2:
        return float("nan")
    return float(np.polyfit(np.log(R[ok]), np.log(y[ok]), 1)[0])


def _batch_run(M, params, fields, steps, chunk, log, label, record_every=None):
    """Advance one batch of droplets `steps` steps (K-step graphs of `chunk`),
    printing progress about every 20 s; returns the sims, their status words
    and step counts, the wall time and, with `record_every`, the history
    [(step, [E_kin of each sim])]: the batch then runs in segments of that
    many steps, closed after each so the members can be read (a diverged
    member leaves the later segments)."""
    import torch
    stream = torch.cuda.Stream()
    sims = []
    with torch.cuda.stream(stream):
        for p, (rR, rB) in zip(params, fields):
            s = M.Sim(p, stream=stream)
            s.init_equilibrium(rR, rB)
            sims.append(s)
    t0 = time.perf_counter()
    seg = steps if not record_every else min(int(record_every), steps)
    counts = [0] * len(sims)
    bad = [False] * len(sims)
    history = []
    done, last = 0, t0
    while done < steps:
        k_seg = min(seg, steps - done)
        alive = [i for i in range(len(sims)) if not bad[i]]
        if not alive:
            break
        batch = M.Batch([sims[i] for i in alive], [k_seg] * len(alive), stream=stream)
        d = 0
        while d < k_seg:
            k = min(chunk, k_seg - d)
            batch.step(k, use_graph=True)   # diverged droplets stop themselves
            d += k
            if time.perf_counter() - last > 20.0:
                stream.synchronize()
                last = time.perf_counter()
                log(f"[sweep] {label}: {done + d}/{steps} steps, {last - t0:.0f} s")
        st, cnt = batch.status()
        batch.close()
        for i, sti, c in zip(alive, st, cnt):
            counts[i] += int(c)
            bad[i] = sti == M.STOPPED_DIVERGED
        done += k_seg
        if record_every:
            history.append((done, [s.observables()["ekin"] if not b else float("nan") for s, b in zip(sims, bad)]))
    status = [M.STOPPED_DIVERGED if b else M.DONE for b in bad]
    out = (sims, status, counts, time.perf_counter() - t0)
    return out + (history,) if record_every else out


def _served_run(M, todo, params, steps, chunk, log):
    """The members as requests of the continuous-batching server (all
    arriving at once); returns their final observables, steps and outcomes
    in `todo` order, and the wall time."""
    from . import serve
    reqs = [serve.Request(i, 0.0, p, "droplet", steps, g, r, SIGMA, radius=float(R))
            for i, ((R, g, r), p) in enumerate(zip(todo, params))]
    server = serve.Server(k_steps=min(chunk, steps), keep_fields=True, policy="shared",
                          log=lambda s: None)
    done, wall = server.run(reqs)
    by = {q.rid: q for q in done}
    out = []
    for i in range(len(todo)):
        q = by[i]
        q.final = None
        out.append((q.obs, q.steps_done, q.outcome, q))
    log(f"[sweep] served {len(todo)} members in {wall:.1f} s")
    return out, wall


def run(study: str, steps: int = 100_000, radii=RADII, chunk: int = 500, log=print, via_server: bool = False):
    """Run one study as a batch (or, via_server, as requests of the sweep
    server, which takes the same steps bit for bit); returns the per-case
    results and the fits."""
    import paper_2110_05197_amd as M
    if study == "ekin":
        return run_ekin(steps=steps, chunk=chunk, log=log)
    if study == "ekin-tau":
        return run_ekin(steps=steps, chunk=chunk, gammas=(1,), taus=EKIN_TAU_R, couplings=(), log=log)
    todo = cases(study, radii)
    params, fields = [], []
    for (R, g, r) in todo:
        p = case_params(M, R, g, r)
        L = p["nx"]
        params.append(p)
        fields.append(inputs.droplet((L, L, L), float(R), p["rho0_R"], p["rho0_B"]))
    results = []
    if via_server:
        served, wall = _served_run(M, todo, params, steps, chunk, log)
        counts = [n for (_, n, _, _) in served]
        for (R, g, r), p, (o, n, outcome, _) in zip(todo, params, served):
            m = measure(o, p, R0=R) if o is not None else dict(R=float("nan"), sigma_cal=float("nan"),
                                                               E=float("nan"), ekin_per_area=float("nan"))
            m.update(R0=R, gamma=g, nu_ratio=r, steps=int(n), diverged=outcome != "done")
            results.append(m)
    else:
        sims, st, counts, wall = _batch_run(M, params, fields, steps, chunk, log, study)
        for (R, g, r), s, p, stat, n in zip(todo, sims, params, st, counts):
            o = s.observables()
            m = measure(o, p, R0=R)
            m.update(R0=R, gamma=g, nu_ratio=r, steps=int(n),
                     diverged=bool(o["diverged"] or stat == M.STOPPED_DIVERGED))
            results.append(m)
            s.close()
    key = "gamma" if study == "density" else "nu_ratio"
    fits = {}
    for v in sorted({m[key] for m in results}):
        sel = [m for m in results if m[key] == v and not m["diverged"]]
        fits[v] = dict(b_E=fit_slope([m["R0"] for m in sel], [m["E"] for m in sel]),
                       b_ekin=fit_slope([m["R0"] for m in sel], [m["ekin_per_area"] for m in sel]),
                       b_E_printed=PRINTED_B[study].get(v if study == "viscosity" else int(v)),
                       b_ekin_printed=PRINTED_B["ekin"].get(int(v)) if study == "density" else None)
    lups = sum(int(n) * p["nx"] ** 3 for p, n in zip(params, counts))
    log(f"[sweep] {study}: {len(todo)} droplets, {steps} steps, {wall:.1f} s, {lups / wall / 1e9:.2f} GLUPS")
    return dict(study=study, steps=steps, wall_s=wall, glups=lups / wall / 1e9, results=results, fits=fits)


# --------------------------------------------------------------------------
# Stationary droplet, CG against SC: spurious-current energy over sigma
# --------------------------------------------------------------------------
EKIN_R = 20
EKIN_SIGMA = (0.001, 0.003, 0.01, 0.03, 0.1, 0.3)
EKIN_GAMMA = (1, 10, 100, 1000)
GSCAN = (-4.4, -4.7, -5.0, -5.3, -5.6, -5.9, -6.2)
EKIN_TAU_R = (0.55, 0.625, 0.75, 0.875, 1.0)
PRINTED_EKIN_B = {"CG": 2.0, "SC": 3.3}
PRINTED_SC_MAX_RATIO = 50.0


def cg_ekin_params(M, gamma, sigma, R=EKIN_R, tau_R=1.0):
    """CG droplet of the E_kin study: FP32 below density ratio 100, FP64 from
    100 on (FP32 storage of the heavy phase's interface populations leaves a
    velocity noise whose energy, at density ratio 1000, exceeds the spurious
    currents of the smaller sigmas and keeps growing with time)."""
    L = box_for(R)
    prec = M.FP64 if gamma >= 100 else M.FP32
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=L, ny=L, nz=L, rho0_R=float(gamma),
                      rho0_B=1.0, tau_R=float(tau_R), tau_B=1.0)
    return M.params_from_sigma(p, sigma)


def sc_ekin_params(M, G, R=EKIN_R):
    """SC multiphase droplet at coupling G, reference densities at the
    flat-interface coexistence pair of G."""
    from .serve import sc_coexistence
    L = box_for(R)
    liq, gas = sc_coexistence(G)
    return M.make_params(lattice=M.D3Q19, model=M.SC_MP, precision=M.FP64, nx=L, ny=L, nz=L, G=float(G),
                         tau_R=1.0, rho0_R=liq, rho0_B=gas)


def sc_pressure(rho, G):
    """Equation of state of the SC multiphase model with psi = 1 - exp(-rho)
    (rho_0 = 1) on a lattice with c_s^2 = 1/3: p = rho/3 + G psi^2 / 6."""
    psi = 1.0 - math.exp(-rho)
    return rho / 3.0 + G * psi * psi / 6.0


def sc_measure(sim, p):
    """rho_in (centre), rho_out (corner), ratio, sigma (Young-Laplace with
    the equimolar radius) and E_kin of an equilibrated SC droplet."""
    rho, _, _ = sim.moments()
    L = p["nx"]
    c = L // 2
    r_in = float(rho[c, c, c])
    r_out = float(rho[0, 0, 0])
    o = sim.observables()
    mass = o["mass_R"]
    dr = r_in - r_out
    R = (3.0 * (mass - r_out * L ** 3) / (4.0 * math.pi * dr)) ** (1.0 / 3.0) if dr > 0 else float("nan")
    dP = sc_pressure(r_in, p["G"]) - sc_pressure(r_out, p["G"])
    return dict(rho_in=r_in, rho_out=r_out, ratio=r_in / r_out if r_out > 0 else float("nan"), R=R,
                sigma=dP * R / 2.0, ekin=o["ekin"], diverged=bool(o["diverged"]))


def settle_step(history, i, tol=0.05):
    """First recorded step from which E_kin of sim i stays within `tol` of
    its last recorded value (the stabilisation of the E_kin-in-time figure
    of section 3.1.2)."""
    final = history[-1][1][i]
    if not final == final or final <= 0:
        return None
    first = None
    for step, ek in history:
        if abs(ek[i] - final) <= tol * final:
            if first is None:
                first = step
        else:
            first = None
    return first


def run_ekin(steps: int = 100_000, chunk: int = 500, sigmas=EKIN_SIGMA, gammas=EKIN_GAMMA, couplings=GSCAN,
             taus=(1.0,), record_every=5000, log=print):
    """The CG and SC stationary droplets as one batch (three groups: CG FP32,
    CG FP64, SC FP64); returns the per-case results and the E_kin fits.
    `taus` lists red relaxation times for the CG droplets (tau_B = 1); with
    more than one, each (density ratio, tau_R) series gets its own fit."""
    import paper_2110_05197_amd as M
    todo, params, fields = [], [], []
    L = box_for(EKIN_R)
    for G in couplings:
        p = sc_ekin_params(M, G)
        rR, rB = inputs.droplet((L, L, L), float(EKIN_R), p["rho0_R"], p["rho0_B"])
        todo.append(("SC", G))
        params.append(p)
        fields.append((rR + rB, None))
    for g in gammas:
        for t in taus:
            for sg in sigmas:
                p = cg_ekin_params(M, g, sg, tau_R=t)
                todo.append(("CG", (g, t, sg)))
                params.append(p)
                fields.append(inputs.droplet((L, L, L), float(EKIN_R), p["rho0_R"], p["rho0_B"]))
    rec = record_every if record_every and steps >= 4 * record_every else None
    res = _batch_run(M, params, fields, steps, chunk, log, "ekin", record_every=rec)
    sims, st, counts, wall = res[:4]
    history = res[4] if rec else []
    sc_rows, cg_rows = [], []
    for idx, ((kind, key), s, p, stat, n) in enumerate(zip(todo, sims, params, st, counts)):
        bad = stat == M.STOPPED_DIVERGED
        if kind == "SC":
            m = sc_measure(s, p) if not bad else dict(diverged=True)
            m.update(G=key, steps=int(n), diverged=bool(bad or m.get("diverged")))
            sc_rows.append(m)
        else:
            o = s.observables()
            m = dict(gamma=key[0], tau_R=key[1], sigma=key[2], ekin=o["ekin"], steps=int(n),
                     diverged=bool(bad or o["diverged"]))
            if history:
                m["settle_step"] = settle_step(history, idx)
                m["ekin_history"] = [(h[0], h[1][idx]) for h in history]
            if not m["diverged"]:
                m["sigma_cal"] = measure(o, p)["sigma_cal"]
            cg_rows.append(m)
        s.close()
    ok_sc = [m for m in sc_rows if not m["diverged"] and m["sigma"] > 0]
    fits = {"SC": dict(b=fit_slope([m["sigma"] for m in ok_sc], [m["ekin"] for m in ok_sc]),
                       b_printed=PRINTED_EKIN_B["SC"],
                       max_ratio=max((m["ratio"] for m in ok_sc), default=float("nan")),
                       max_ratio_printed=PRINTED_SC_MAX_RATIO)}
    for g in gammas:
        for t in taus:
            sel = [m for m in cg_rows if m["gamma"] == g and m["tau_R"] == t and not m["diverged"]]
            name = f"CG gamma={g}" if len(taus) == 1 else f"CG gamma={g} tau_R={t}"
            fits[name] = dict(b=fit_slope([m["sigma"] for m in sel], [m["ekin"] for m in sel]),
                              b_printed=PRINTED_EKIN_B["CG"], n=len(sel))
    lups = sum(int(n) * p["nx"] ** 3 for p, n in zip(params, counts))
    log(f"[sweep] ekin: {len(todo)} droplets, {steps} steps, {wall:.1f} s, {lups / wall / 1e9:.2f} GLUPS")
    return dict(study="ekin", steps=steps, wall_s=wall, glups=lups / wall / 1e9, sc=sc_rows, cg=cg_rows,
                fits=fits)
