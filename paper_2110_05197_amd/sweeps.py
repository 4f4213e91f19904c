"""Parameter sweeps of the paper's static-droplet studies, run as one batch of
independent simulations on the GPU (the batch API of the library).

Study "density" (Laplace test, section 3.1): a 3-D colour-gradient droplet of
radius R = 8, 12, 16, 20 at density ratios rho_R/rho_B = 1, 10, 100, 1000 and
viscosity ratio 1; study "viscosity": density ratio 1 and viscosity ratios
nu_R/nu_B = 1, 2, 5, 10, 100.  sigma_th = 0.01 throughout (Eq. sigmaA).  After
the equilibration each droplet gives

* sigma_cal from Young-Laplace in 3-D, dP = 2 sigma / R (Eq. YoungLaplace),
  with p_k = rho_k (1 - alpha_k) / 2 (the sound speed of colour k on D3Q19,
  Eq. gamma) from the epsilon-masked inside/outside densities and R the
  equimolar radius of the red mass, (3 M_R / (4 pi rho_in))^(1/3) (reading:
  the red volume sum (1 + rho^N)/2 puts the interface at rho^N = 0, which at a
  density ratio lies far out on the light side);
* the error E = |sigma_th - sigma_cal| / sigma_th;
* the kinetic energy of the spurious currents per droplet area,
  E_kin / (4 pi R^2);

and each series is fitted with E ∝ R^b and E_kin / A_d ∝ R^b, the fits the
paper tabulates (Tables densErrors, viscErrors, radiusErrors).

Readings: rho_B = 1 and rho_R = gamma (as for the other density-ratio cases);
the viscosity ratio r is split as nu_R = nu0 sqrt(r), nu_B = nu0 / sqrt(r)
with nu0 = 1/6, so that every tau stays in [0.55, 5.5]; the box is periodic,
L = 4 R + 16 (multiple of 8), the droplet centred; mixed precision (FP64 sums
and light-phase arithmetic) for density ratios >= 100, FP32 otherwise.
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


def box_for(R: int) -> int:
    return int(math.ceil((4 * R + 16) / 8.0) * 8)


def case_params(M, R, gamma, nu_ratio):
    L = box_for(R)
    nu0 = 1.0 / 6.0
    nuR, nuB = nu0 * math.sqrt(nu_ratio), nu0 / math.sqrt(nu_ratio)
    prec = M.MIXED if gamma >= 100 else M.FP32
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=L, ny=L, nz=L, rho0_R=float(gamma),
                      rho0_B=1.0, tau_R=0.5 + 3 * nuR, tau_B=0.5 + 3 * nuB)
    return M.params_from_sigma(p, SIGMA)


def cases(study: str, radii=RADII):
    if study == "density":
        return [(R, g, 1.0) for g in (1, 10, 100, 1000) for R in radii]
    if study == "viscosity":
        return [(R, 1, r) for r in (1, 2, 5, 10, 100) for R in radii]
    raise ValueError(study)


def measure(obs, p):
    """sigma_cal, E and E_kin / A_d of one equilibrated droplet."""
    aR = 1.0 - (1.0 - p["alpha_B"]) * p["rho0_B"] / p["rho0_R"]   # Eq. gamma
    cR2, cB2 = (1.0 - aR) / 2.0, (1.0 - p["alpha_B"]) / 2.0
    R = (3.0 * obs["mass_R"] / (4.0 * math.pi * obs["rho_in"])) ** (1.0 / 3.0)
    R_vol = (3.0 * obs["red_volume"] / (4.0 * math.pi)) ** (1.0 / 3.0)
    dP = obs["rho_in"] * cR2 - obs["rho_out"] * cB2
    sigma_cal = dP * R / 2.0
    return dict(R=R, R_red_volume=R_vol, sigma_cal=sigma_cal, E=abs(SIGMA - sigma_cal) / SIGMA,
                ekin_per_area=obs["ekin"] / (4.0 * math.pi * R * R), eps=obs["eps_used"])


def fit_slope(R, y):
    R, y = np.asarray(R, float), np.asarray(y, float)
    ok = y > 0
    if ok.sum() < 2:
        return float("nan")
    return float(np.polyfit(np.log(R[ok]), np.log(y[ok]), 1)[0])


def run(study: str, steps: int = 100_000, radii=RADII, chunk: int = 500, log=print):
    """Run one study as a batch; returns the per-case results and the fits."""
    import torch
    import paper_2110_05197_amd as M
    todo = cases(study, radii)
    stream = torch.cuda.Stream()
    sims, params = [], []
    with torch.cuda.stream(stream):
        for (R, g, r) in todo:
            p = case_params(M, R, g, r)
            L = p["nx"]
            rR, rB = inputs.droplet((L, L, L), float(R), p["rho0_R"], p["rho0_B"])
            s = M.Sim(p, stream=stream)
            s.init_equilibrium(rR, rB)
            sims.append(s)
            params.append(p)
    t0 = time.perf_counter()
    batch = M.Batch(sims, [steps] * len(sims), stream=stream)
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        batch.step(k, use_graph=True)   # diverged droplets stop themselves
        done += k
    st, counts = batch.status()
    batch.close()
    wall = time.perf_counter() - t0
    results = []
    for (R, g, r), s, p, stat, n in zip(todo, sims, params, st, counts):
        o = s.observables()
        m = measure(o, p)
        m.update(R0=R, gamma=g, nu_ratio=r, steps=int(n), diverged=bool(o["diverged"] or stat == M.STOPPED_DIVERGED))
        results.append(m)
        s.close()
    key = "gamma" if study == "density" else "nu_ratio"
    fits = {}
    for v in sorted({m[key] for m in results}):
        sel = [m for m in results if m[key] == v and not m["diverged"]]
        fits[v] = dict(b_E=fit_slope([m["R"] for m in sel], [m["E"] for m in sel]),
                       b_ekin=fit_slope([m["R"] for m in sel], [m["ekin_per_area"] for m in sel]),
                       b_E_printed=PRINTED_B[study].get(v if study == "viscosity" else int(v)),
                       b_ekin_printed=PRINTED_B["ekin"].get(int(v)) if study == "density" else None)
    lups = sum(int(n) * p["nx"] ** 3 for p, n in zip(params, counts))
    log(f"[sweep] {study}: {len(todo)} droplets, {steps} steps, {wall:.1f} s, {lups / wall / 1e9:.2f} GLUPS")
    return dict(study=study, steps=steps, wall_s=wall, glups=lups / wall / 1e9, results=results, fits=fits)
