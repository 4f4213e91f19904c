"""Physics runs of the paper's breakup and high-density-ratio cases on the GPU,
reporting the quantities the paper measures on them.

* ``rayleigh_plateau(model)``: the periodic jet of the breakup section
  (128 x 128 x 512, axis along z, R0 = 12, sinusoidal radius perturbation of
  0.1 R0, wavelength drawn in [9 R0, 12 R0] and made commensurate with the
  box), colour gradient or two-component Shan-Chen at density ratio 1, FP32,
  the colour-gradient sigma set to the Shan-Chen one measured by
  ``sc_mc_sigma`` (matched surface tension).
  Every ``every`` steps the droplet counter gives the number of droplets and
  their node counts: the breakup time is the first sample with more than one
  droplet; satellites are the droplets below a quarter of the largest; their
  node count over time shows whether they keep their mass (CG) or dissolve
  into the other component (SC).
* ``sc_mc_sigma(G_RB)``: surface tension of the two-component Shan-Chen model
  from a Laplace test, dP = 2 sigma / R (Eq. YoungLaplace), with the pressure
  p = (rho_R + rho_B) / 3 + (G_RB / rho0_X^2) rho_R rho_B / 3 of the cross
  force (Eq. doublebeltrepulsionforce2 on belt 1) and R from the rho^N = 0
  crossings along x through the centre.
* ``ligament_contraction()``: the capsules of Table contrParams (128 x 64 x
  64 periodic, sets 1-4, plus set 1 without the enhanced equilibrium), the
  endpoint speed after start-up against sqrt(sigma / (rho_R R0)).
* ``ligament(precision)``: the high-density-ratio capsule (96 x 96 x 384,
  walls on x and y, outflow on z, R0 = 8, length 320, density ratio 1000,
  viscosity ratio 50, sigma = 0.01); the end positions from the interface
  crossings along z near the axis, the retraction speed of each end against
  the capillary speed sqrt(sigma / (rho_R R0)) of the contraction section,
  the droplet count and divergence.
* ``mass_drift(params, fields)``: how each colour's total mass moves under
  reduced-precision storage (exact in FP64) over many steps, sampled every
  ``every`` steps, with the exponent b of |drift| ~ t^b fitted over the later
  samples (b = 1: a bias that accumulates at a steady rate; b = 1/2: a random
  walk of the per-step rounding) and how often the drift keeps its sign.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs

RP_R0 = 12.0
RP_SHAPE = (512, 128, 128)


def rp_wavelength(seed: int = 3):
    """Wavelength in [9 R0, 12 R0] made commensurate with the 512-node axis,
    and a phase, from the seed."""
    rng = np.random.default_rng(seed)
    lam = 512 / round(512 / rng.uniform(9 * RP_R0, 12 * RP_R0))
    return lam, float(rng.uniform(0, 2 * math.pi))


# Two-component Shan-Chen at density ratio 1: coupling SC_G, total density
# SC_TOTAL per node; each phase holds its majority species at a and the other
# species dissolved at b, the coexisting pair of the cross force with psi =
# rho (equal chemical potentials ln rho_s + G rho_s' of both species in both
# phases, which by symmetry leaves ln(a / b) = G (a - b), a + b = SC_TOTAL).
# The 50/50 mixture is unstable to demixing since G_RB SC_TOTAL / 2 > 1.
SC_G, SC_TOTAL = 1.5, 2.0


def sc_mc_coexistence(G: float = SC_G, total: float = SC_TOTAL):
    """(majority, minority) densities of the demixed phases."""
    from scipy.optimize import brentq
    h = total / 2.0
    g = lambda d: math.log((h + d) / (h - d)) - G * 2.0 * d
    if G * h <= 1.0:
        raise ValueError("the mixture does not demix: G_RB * total / 2 <= 1")
    d = brentq(g, 1e-9 * h, h * (1 - 1e-12))
    return h + d, h - d


SC_RHO, SC_MINOR = sc_mc_coexistence()


def rp_params(M, model: str, sigma: float = 0.03):
    nz, ny, nx = RP_SHAPE
    if model == "CG":
        p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=nx, ny=ny, nz=nz)
        return M.params_from_sigma(p, sigma)
    return M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=nx, ny=ny, nz=nz,
                         G_RB=SC_G, rho0_R=SC_RHO, rho0_B=SC_RHO)


def rp_fields(model: str, seed: int = 3):
    lam, phase = rp_wavelength(seed)
    if model == "CG":
        rR, rB = inputs.jet(RP_SHAPE, RP_R0, lam, 0.1, phase)
    else:
        rR, rB = inputs.jet(RP_SHAPE, RP_R0, lam, 0.1, phase, SC_RHO - SC_MINOR, SC_RHO - SC_MINOR)
        rR, rB = rR + SC_MINOR, rB + SC_MINOR
    return rR, rB, lam


def rayleigh_plateau(M, model: str, steps: int = 30000, every: int = 500, seed: int = 3, sigma: float = 0.03,
                     log=print):
    """sigma: the colour-gradient surface tension (Eq. sigmaA); pass the
    Shan-Chen one to compare the two at matched sigma."""
    p = rp_params(M, model, sigma)
    rR, rB, lam = rp_fields(model, seed)
    s = M.Sim(p)
    s.init_equilibrium(rR, rB)
    history = []
    t0 = time.perf_counter()
    done = 0
    status = M.OK
    while done < steps:
        st, k = s.step(min(every, steps - done), check_every=every)
        done += k
        n, sizes = s.droplets(64)
        history.append((done, n, sizes[:16]))
        if st != M.OK:
            status = st
            break
    wall = time.perf_counter() - t0
    s.close()
    breakup = next((t for t, n, _ in history if n > 1), None)
    sat = []
    for t, n, sizes in history:
        if n > 1:
            big = sizes[0]
            sat.append((t, sum(v for v in sizes if v < 0.25 * big), sum(1 for v in sizes if v < 0.25 * big),
                        sum(1 for v in sizes if v >= 0.25 * big)))
    out = dict(model=model, wavelength=lam, wavelengths_in_box=round(512 / lam), steps=done,
               diverged=status != M.OK, breakup_step=breakup, wall_s=round(wall, 1),
               glups=round(done * 512 * 128 * 128 / wall / 1e9, 2),
               final_count=history[-1][1], final_sizes=history[-1][2],
               satellites=[dict(step=t, nodes=m, count=c, main=mc) for t, m, c, mc in sat])
    log(f"[rp] {model}: breakup at step {breakup}, final {history[-1][1]} droplets {history[-1][2][:8]}")
    return out


def sc_mc_sigma(M, G_RB: float = SC_G, R: float = 16.0, L: int = 64, steps: int = 8000):
    """Laplace-test surface tension of the two-component Shan-Chen model."""
    p = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=L, ny=L, nz=L, G_RB=G_RB,
                      rho0_R=SC_RHO, rho0_B=SC_RHO)
    rR, rB = inputs.droplet((L, L, L), R, SC_RHO - SC_MINOR, SC_RHO - SC_MINOR)
    s = M.Sim(p)
    s.init_equilibrium(rR + SC_MINOR, rB + SC_MINOR)
    st, _ = s.step(steps, check_every=steps)
    c = L // 2
    xs, n = s.interface_crossings(0, c, c)
    mR, mB, _ = s.moments()
    mR, mB = mR.cpu().numpy(), mB.cpu().numpy()
    s.close()
    xpref = G_RB / p["rho0_X"] ** 2
    pres = lambda a, b: (a + b) / 3.0 + xpref * a * b / 3.0
    inside = (slice(c - 1, c + 1),) * 3
    p_in = float(np.mean(pres(mR[inside], mB[inside])))
    p_out = float(pres(mR[0, 0, 0], mB[0, 0, 0]))
    radius = (xs[-1] - xs[0]) / 2.0 if n >= 2 else float("nan")
    return dict(G_RB=G_RB, sigma=(p_in - p_out) * radius / 2.0, radius=radius, dP=p_in - p_out,
                rho_in=(float(np.mean(mR[inside])), float(np.mean(mB[inside]))),
                rho_out=(float(mR[0, 0, 0]), float(mB[0, 0, 0])), status_ok=st == M.OK)


LIG_SHAPE = (384, 96, 96)


def ligament(M, precision, steps: int = 40000, every: int = 2000, log=print):
    nz, ny, nx = LIG_SHAPE
    R0, length, sigma = 8.0, 320.0, 0.01
    rR, rB = inputs.ligament(LIG_SHAPE, R0, length, 1000.0, 1.0, axis=2)
    p = M.make_params(lattice=M.D3Q19, precision=precision, nx=nx, ny=ny, nz=nz, bc=(1, 1, 2),
                      rho0_R=1000.0, rho0_B=1.0, tau_R=3.0, tau_B=0.55)
    p = M.params_from_sigma(p, sigma)
    s = M.Sim(p)
    s.init_equilibrium(rR, rB)
    cx, cy = nx // 2, ny // 2
    ends = []
    status = M.OK
    done = 0
    t0 = time.perf_counter()
    while True:
        xs, n = s.interface_crossings(2, cx, cy)
        ends.append((done, xs[0] if n else float("nan"), xs[-1] if n else float("nan"), n))
        if done >= steps:
            break
        st, k = s.step(min(every, steps - done), check_every=every)
        done += k
        if st != M.OK:
            status = st
            xs, n = s.interface_crossings(2, cx, cy)
            ends.append((done, xs[0] if n else float("nan"), xs[-1] if n else float("nan"), n))
            break
    wall = time.perf_counter() - t0
    count, sizes = s.droplets(16)
    obs = s.observables()
    s.close()
    t = np.array([e[0] for e in ends], float)
    lo = np.array([e[1] for e in ends])
    hi = np.array([e[2] for e in ends])
    # retraction speed of each end over the second half of the run
    sel = t >= t[-1] / 2
    v_lo = float(np.polyfit(t[sel], lo[sel], 1)[0]) if sel.sum() >= 2 else float("nan")
    v_hi = float(-np.polyfit(t[sel], hi[sel], 1)[0]) if sel.sum() >= 2 else float("nan")
    u_cap = math.sqrt(sigma / (1000.0 * R0))
    out = dict(precision=precision, steps=done, diverged=status != M.OK or bool(obs["diverged"]),
               length=[round(h - l, 2) for l, h in zip(lo, hi)], steps_sampled=[int(x) for x in t],
               end_speed=(v_lo, v_hi), capillary_speed=u_cap, speed_ratio=((v_lo + v_hi) / 2) / u_cap,
               final_count=count, final_sizes=sizes[:4], wall_s=round(wall, 1),
               mass_R=obs["mass_R"], mass_B=obs["mass_B"])
    log(f"[ligament] precision {precision}: {done} steps, length {out['length'][0]} -> {out['length'][-1]}, "
        f"end speed {out['speed_ratio']:.2f} x sqrt(sigma/(rho_R R0)), {count} droplet(s)")
    return out


# ---------------------------------------------------------------------------
# Ligament contraction (Table contrParams, sets 1-4)
# ---------------------------------------------------------------------------
CONTR_SHAPE = (64, 64, 128)     # (nz, ny, nx): 128 x 64 x 64 periodic, axis along x
CONTR_SETS = (
    dict(name="1", model="CG", rho=(2.0, 0.1), tau=(1.0, 0.55), sigma=0.05, R0=12.0, L=112.0, enhanced=1),
    dict(name="1 plain", model="CG", rho=(2.0, 0.1), tau=(1.0, 0.55), sigma=0.05, R0=12.0, L=112.0, enhanced=0),
    dict(name="2", model="CG", rho=(1.99, 0.165), tau=(1.0, 1.0), sigma=0.078, R0=10.0, L=100.0, enhanced=1),
    dict(name="3", model="SC", G=-5.0, tau=(1.0,), R0=10.0, L=100.0),
    dict(name="2 matched", model="CG", match_sc=True, G=-5.0, tau=(1.0, 1.0), R0=10.0, L=100.0, enhanced=1),
    dict(name="4", model="CG", rho=(1.99, 0.165), tau=(1.0, 0.55), sigma=0.078, R0=10.0, L=100.0, enhanced=1),
)


def sc_mp_sigma(M, G: float, R: int = 16, steps: int = 20000):
    """Surface tension and the drop/vapour densities of the SC multiphase model
    at coupling G: a droplet of radius R in the 64^3 Laplace box, started at
    the flat coexistence pair, Young-Laplace with p = rho/3 + G psi^2/6."""
    from . import sweeps
    p = sweeps.sc_ekin_params(M, G, R=R)
    L = p["nx"]
    rR, rB = inputs.droplet((L, L, L), float(R), p["rho0_R"], p["rho0_B"])
    s = M.Sim(p)
    s.init_equilibrium(rR + rB, None)
    s.step(steps)
    m = sweeps.sc_measure(s, p)
    s.close()
    return m


def contraction_scales(rho_R: float, sigma: float, R0: float, L: float, tau_R: float):
    """Capillary time sqrt(rho_R R0^3 / sigma), Srivastava end speed
    sqrt(sigma / (rho_R R0)) and Ohnesorge number mu / sqrt(rho_R sigma L)
    with mu = rho_R (tau_R - 1/2) / 3, as the contraction section defines them."""
    mu = rho_R * (tau_R - 0.5) / 3.0
    return (math.sqrt(rho_R * R0 ** 3 / sigma), math.sqrt(sigma / (rho_R * R0)),
            mu / math.sqrt(rho_R * sigma * L))


def contraction_run(M, cfg: dict, span: float = 4.5, fit=(2.0, 4.0)):
    """One ligament of Table contrParams (FP64): the capsule of radius R0 and
    length L along x, its endpoint x_e(t) from the outermost interface
    crossing on the axis, sampled about 30 times per capillary time
    t_cap = sqrt(rho_R R0^3 / sigma) up to `span` t_cap; the endpoint speed is
    the slope over t / t_cap in `fit`, divided by the Srivastava speed
    sqrt(sigma / (rho_R R0)) of the contraction section."""
    nz, ny, nx = CONTR_SHAPE
    R0, length = cfg["R0"], cfg["L"]
    if cfg["model"] == "SC":
        m = sc_mp_sigma(M, cfg["G"])
        rhoR, rhoB, sigma = m["rho_in"], m["rho_out"], m["sigma"]
        p = M.make_params(lattice=M.D3Q19, model=M.SC_MP, precision=M.FP64, nx=nx, ny=ny, nz=nz,
                          G=cfg["G"], tau_R=cfg["tau"][0], rho0_R=rhoR, rho0_B=rhoB)
        rR, rB = inputs.ligament(CONTR_SHAPE, R0, length, rhoR, rhoB, axis=0)
        fields = (rR + rB, None)
    else:
        if cfg.get("match_sc"):      # sigma and densities of the SC model at this G
            m = sc_mp_sigma(M, cfg["G"])
            rhoR, rhoB, sigma = m["rho_in"], m["rho_out"], m["sigma"]
        else:
            (rhoR, rhoB), sigma = cfg["rho"], cfg["sigma"]
        p = M.make_params(lattice=M.D3Q19, precision=M.FP64, nx=nx, ny=ny, nz=nz, rho0_R=rhoR, rho0_B=rhoB,
                          tau_R=cfg["tau"][0], tau_B=cfg["tau"][1], enhanced_eq=cfg["enhanced"])
        p = M.params_from_sigma(p, sigma)
        fields = inputs.ligament(CONTR_SHAPE, R0, length, rhoR, rhoB, axis=0)
    tcap, u_an, Oh = contraction_scales(rhoR, sigma, R0, length, cfg["tau"][0])
    every = max(2, int(round(tcap / 30.0)))
    s = M.Sim(p)
    s.init_equilibrium(*fields)
    ts, xe, status = [], [], M.OK
    for k in range(int(span * tcap / every)):
        st, _ = s.step(every, check_every=every)
        if st != M.OK:
            status = st
            break
        pos, n = s.interface_crossings(0, ny // 2, nz // 2)
        if n < 2:
            break
        ts.append((k + 1) * every / tcap)
        xe.append((pos[-1] - (nx - 1) / 2.0) / R0)
    s.close()
    ts, xe = np.array(ts), np.array(xe)
    sel = (ts >= fit[0]) & (ts <= fit[1])
    speed = -float(np.polyfit(ts[sel], xe[sel], 1)[0]) if sel.sum() >= 3 else float("nan")
    return dict(set=cfg["name"], model=cfg["model"], rho_R=rhoR, rho_B=rhoB, sigma=sigma, R0=R0, L=length,
                tau=cfg["tau"], t_cap=tcap, u_analytic=u_an, speed_ratio=speed, Oh=Oh, diverged=status != M.OK,
                t=[round(x, 3) for x in ts[::3]], x_end=[round(x, 4) for x in xe[::3]])


def ligament_contraction(M, sets=CONTR_SETS, log=print):
    """Every set of Table contrParams (plus set 1 without the enhanced
    equilibrium, and set 2 re-run at the surface tension and densities the
    SC model of set 3 actually has here, for a matched CG-SC pair)."""
    out = []
    for cfg in sets:
        r = contraction_run(M, cfg)
        log(f"[contraction] set {r['set']} ({r['model']}): sigma {r['sigma']:.4f}, rho {r['rho_R']:.3f}/"
            f"{r['rho_B']:.3f}, Oh {r['Oh']:.3f}, t_cap {r['t_cap']:.1f}: endpoint speed "
            f"{r['speed_ratio']:.3f} x sqrt(sigma/(rho_R R0))")
        out.append(r)
    return out


# ---------------------------------------------------------------------------
# Oscillating droplet (the droplet-oscillation section; l = 2 shape mode)
# ---------------------------------------------------------------------------
def lamb_omega(sigma: float, R: float, rho_in: float = 1.0, rho_out: float = 1.0) -> float:
    """Inviscid l = 2 frequency of a drop in a host fluid."""
    return math.sqrt(24.0 * sigma / (R ** 3 * (3.0 * rho_in + 2.0 * rho_out)))


def miller_scriven_omega(sigma, R, rho_in, rho_out, nu_in, nu_out):
    """Lamb's frequency with the first viscous corrections of Miller and
    Scriven (Eqs. millscriv-millscriv3)."""
    den = 3.0 * rho_in + 2.0 * rho_out
    w = lamb_omega(sigma, R, rho_in, rho_out)
    a = (25.0 * math.sqrt(nu_in * nu_out) * rho_in * rho_out
         / (math.sqrt(2.0) * R * den * (math.sqrt(nu_in) * rho_in + math.sqrt(nu_out) * rho_out)))
    return w - 0.5 * a * math.sqrt(w) + 0.25 * a * a


def fit_damped_cosine(t, r, w0):
    """R(t) = R_D + b exp(-l t) cos(w t + ph) by least squares; (w, l, R_D)."""
    from scipy.optimize import curve_fit
    model = lambda t, a, b, lam, w, ph: a + b * np.exp(-lam * t) * np.cos(w * t + ph)
    best = None
    for wf in (1.0, 0.7, 1.4):                     # start near, below and above the expected w
        for ph0 in (0.0, math.pi / 2, math.pi, 3 * math.pi / 2):
            try:
                pp, _ = curve_fit(model, t, r, p0=[float(r.mean()), float(r[0] - r.mean()), 1e-4, wf * w0, ph0],
                                  maxfev=20000)
            except RuntimeError:
                continue
            if pp[2] < 0:                          # a growing envelope is no damped oscillation
                continue
            res = float(np.sum((model(t, *pp) - r) ** 2))
            if best is None or res < best[0]:
                best = (res, pp)
    if best is None:
        return float("nan"), float("nan"), float("nan")
    pp = best[1]
    return abs(float(pp[3])), float(pp[2]), float(pp[0])


def oscillation(M, precision, n: int = 128, steps: int = 20000, every: int = 20, seed: int = 2, log=print):
    """Ellipsoid with semi-axes (24, 20, 20), each perturbed by U[-1, 1], tau
    from U[0.55, 1.0], A = 0.005, density and viscosity ratio 1, n^3
    periodic: the y-axis radius from the interface crossings every `every`
    steps, its damped-cosine frequency against Lamb's and Miller-Scriven's."""
    rng = np.random.default_rng(seed)
    tau = float(rng.uniform(0.55, 1.0))
    (rR, rB), axes = inputs.perturbed_ellipsoid((n, n, n), (24.0, 20.0, 20.0), seed=seed)
    p = M.make_params(lattice=M.D3Q19, precision=precision, nx=n, ny=n, nz=n, A=0.005, tau_R=tau, tau_B=tau)
    s = M.Sim(p)
    s.init_equilibrium(rR, rB)
    c = n // 2
    t, r = [], []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        st, k = s.step(every, check_every=every)
        done += k
        xs, cnt = s.interface_crossings(1, c, c)
        t.append(done)
        r.append((xs[-1] - xs[0]) / 2.0 if cnt >= 2 else float("nan"))
        if st != M.OK:
            break
    wall = time.perf_counter() - t0
    o = s.observables()
    s.close()
    t, r = np.array(t, float), np.array(r)
    sigma = M.sigma_from_params(p)
    RD = (3.0 * o["red_volume"] / (4.0 * math.pi)) ** (1.0 / 3.0)
    nu = (tau - 0.5) / 3.0
    wL = lamb_omega(sigma, RD)
    wMS = miller_scriven_omega(sigma, RD, 1.0, 1.0, nu, nu)
    ok = np.isfinite(r)
    w, lam, rfit = fit_damped_cosine(t[ok], r[ok], wMS)
    out = dict(precision=precision, tau=tau, axes=[float(a) for a in axes], sigma=sigma, R_D=RD, steps=done,
               omega=w, damping=lam, period=2 * math.pi / w if w == w and w > 0 else float("nan"),
               omega_lamb=wL, omega_miller_scriven=wMS, err_vs_lamb=(w - wL) / wL, err_vs_ms=(w - wMS) / wMS,
               wall_s=round(wall, 1), radius_first=float(r[0]), radius_last=float(r[-1]))
    log(f"[oscillation] precision {precision} tau={tau:.3f} R_D={RD:.2f}: period {out['period']:.0f} steps, "
        f"omega {w:.4e} vs Lamb {wL:.4e} ({out['err_vs_lamb']:+.1%}), Miller-Scriven {wMS:.4e} "
        f"({out['err_vs_ms']:+.1%})")
    return out


# ---------------------------------------------------------------------------
# Oscillating droplet at the parameters of Table dropOscParams
# ---------------------------------------------------------------------------
OSC_RHO = (2.73, 0.073)
OSC_SIGMA = 0.183
OSC_RADII = (12, 25, 37, 49)
PRINTED_DROPOSC = {   # Table dropOsc: (R_D, omega_2, E in %)
    "CG": ((11.65, 14.65e-3, 11.51), (24.97, 5.20e-3, 2.49), (36.97, 2.97e-3, 0.31), (48.95, 1.96e-3, 0.16)),
    "SC": ((11.79, 1.17e-3, 27.96), (24.62, 4.44e-3, 15.45), (37.02, 2.62e-3, 10.52), (48.60, 1.94e-3, 7.77)),
}


def osc_box(R: float):
    """(nz, ny, nx): the 160 x 160 x 240 box of the oscillation section, long
    axis along z; 240 x 240 x 360 from R_D = 49 on (the section enlarges the
    box there to keep the droplet clear of its periodic images)."""
    return (360, 240, 240) if R >= 45 else (240, 160, 160)


def oscillation_run(M, model: str, R: float, periods: float = 5.0, aspect: float = 1.25, sigma=None, beta=None,
                    log=print):
    """One droplet of Table dropOscParams (FP64, tau = 1 in both phases): a
    prolate ellipsoid of volume (4/3) pi R^3 and axis ratio `aspect` along z,
    its y-axis radius R(t) through the box centre from the interface crossings
    (rho^N = 0 for CG, the mid density for SC) about 40 times per period, the
    damped-cosine fit R(t) = R_D + b exp(-l t) cos(w t + ph), and the error of
    w against Miller-Scriven (Eqs. millscriv-millscriv3) at the fitted R_D.

    CG: rho 2.73 / 0.073, sigma 0.183 (or `sigma`), recolouring beta 0.7 (or
    `beta`).  SC (multiphase): the coupling whose
    coexistence has the same density ratio (37.4), densities and sigma from a
    Laplace run of that model (the paper's G = -6 maps to other densities in
    its pseudopotential, R17)."""
    from .serve import sc_coupling_for_ratio
    shape = osc_box(R)
    nz, ny, nx = shape
    a = R / aspect ** (1.0 / 3.0)
    axes = (a, a, a * aspect)
    if model == "SC":
        G = sc_coupling_for_ratio(OSC_RHO[0] / OSC_RHO[1])
        m = sc_mp_sigma(M, G)
        rho_in, rho_out, sigma = m["rho_in"], m["rho_out"], m["sigma"]
        p = M.make_params(lattice=M.D3Q19, model=M.SC_MP, precision=M.FP64, nx=nx, ny=ny, nz=nz, G=G,
                          tau_R=1.0, rho0_R=rho_in, rho0_B=rho_out)
        rR, rB = inputs.ellipsoid(shape, axes, rho_in, rho_out)
        fields = (rR + rB, None)
    else:
        G = None
        (rho_in, rho_out), sigma = OSC_RHO, (OSC_SIGMA if sigma is None else sigma)
        p = M.make_params(lattice=M.D3Q19, precision=M.FP64, nx=nx, ny=ny, nz=nz, rho0_R=rho_in,
                          rho0_B=rho_out, tau_R=1.0, tau_B=1.0)
        if beta is not None:
            p["beta"] = float(beta)
        p = M.params_from_sigma(p, sigma)
        fields = inputs.ellipsoid(shape, axes, rho_in, rho_out)
    nu = 1.0 / 6.0
    w_guess = miller_scriven_omega(sigma, R, rho_in, rho_out, nu, nu)
    period = 2.0 * math.pi / w_guess
    every = max(2, int(round(period / 40.0)))
    steps = int(periods * period)
    s = M.Sim(p)
    s.init_equilibrium(*fields)
    t, r, status = [], [], M.OK
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        st, k = s.step(every, check_every=every)
        done += k
        if st != M.OK:
            status = st
            break
        xs, cnt = s.interface_crossings(1, nx // 2, nz // 2)
        t.append(done)
        r.append((xs[-1] - xs[0]) / 2.0 if cnt >= 2 else float("nan"))
    wall = time.perf_counter() - t0
    s.close()
    t, r = np.array(t, float), np.array(r)
    ok = np.isfinite(r) & (t >= 0.25 * period)      # leave out the interface's first settling
    if ok.sum() >= 20:
        w, lam, RD = fit_damped_cosine(t[ok], r[ok], w_guess)
    else:
        w = lam = RD = float("nan")
    w_ms = miller_scriven_omega(sigma, RD, rho_in, rho_out, nu, nu) if RD == RD else float("nan")
    label = model if model == "SC" else "CG" + (f" sigma={sigma}" if sigma is not None else "") + (
        f" beta={beta}" if beta is not None else "")
    out = dict(model=label, R=R, box=[nx, ny, nz], G=G, rho_in=rho_in, rho_out=rho_out, sigma=sigma,
               steps=done, every=every, R_D=RD, omega=w, damping=lam, omega_ms=w_ms,
               E=abs(w_ms - w) / w_ms, diverged=status != M.OK, wall_s=round(wall, 1))
    log(f"[oscillation] {out['model']} R={R}: R_D {RD:.2f}, omega {w:.4e} vs Miller-Scriven {w_ms:.4e}: "
        f"E {100 * out['E']:.2f} %  ({done} steps, {wall:.0f} s{', diverged' if out['diverged'] else ''})")
    return out


def oscillation_table(M, radii=OSC_RADII, models=("CG", "SC"), cg_sigmas=(0.05,), cg_betas=(0.5,), log=print):
    """Table dropOsc re-run: every model at every radius, with the printed
    values beside the measured ones; then the CG droplets again at each of
    `cg_sigmas` (same densities and tau), below the printed sigma, and at the
    printed sigma with each recolouring beta of `cg_betas`."""
    rows = []
    for model in models:
        for R in radii:
            o = oscillation_run(M, model, float(R), log=log)
            pr = PRINTED_DROPOSC[model][OSC_RADII.index(R)] if R in OSC_RADII else None
            o["printed"] = dict(R_D=pr[0], omega=pr[1], E_percent=pr[2]) if pr else None
            rows.append(o)
    for sg in cg_sigmas:
        for R in radii:
            rows.append(oscillation_run(M, "CG", float(R), sigma=sg, log=log))
    for b in cg_betas:
        for R in radii:
            rows.append(oscillation_run(M, "CG", float(R), beta=b, log=log))
    return rows


def mass_drift(M, params: dict, rR, rB, steps: int = 10000, every: int = 250, log=print):
    """Relative change of each colour's total mass every `every` steps over
    `steps` steps of one lattice, and its growth law (see the module notes)."""
    sim = M.Sim(params)
    sim.init_equilibrium(rR, rB)
    o0 = sim.observables()
    ts, dR, dB = [], [], []
    t0 = time.perf_counter()
    for s in range(every, steps + 1, every):
        st, _ = sim.step(every, check_every=every)
        if st != M.OK:
            break
        o = sim.observables()
        ts.append(s)
        dR.append((o["mass_R"] - o0["mass_R"]) / o0["mass_R"])
        dB.append((o["mass_B"] - o0["mass_B"]) / o0["mass_B"])
        if s % (every * 8) == 0:
            log(f"[drift] step {s}: red {dR[-1]:+.3e}, blue {dB[-1]:+.3e}")
    wall = time.perf_counter() - t0
    sim.close()
    t = np.array(ts, dtype=float)

    def law(d):
        d = np.array(d)
        late = (t >= t[-1] / 10) & (np.abs(d) > 0)
        b = float(np.polyfit(np.log(t[late]), np.log(np.abs(d[late])), 1)[0]) if late.sum() >= 3 else float("nan")
        same = float(np.mean(np.sign(d[late]) == np.sign(d[-1]))) if late.any() else float("nan")
        return dict(final=float(d[-1]), per_step=float(d[-1] / t[-1]), exponent=b, same_sign_fraction=same)

    return dict(steps=int(t[-1]) if len(t) else 0, every=every, wall_s=round(wall, 1),
                red=law(dR), blue=law(dB), series=dict(step=ts, red=dR, blue=dB))
