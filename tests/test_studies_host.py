"""Host-side pieces of the physics studies: the two-component Shan-Chen
coexistence pair used to initialise the breakup runs, checked against the
oracle, and the Lamb / Miller-Scriven frequencies against their limits."""
import math

import numpy as np
import pytest

from paper_2110_05197_amd import studies


def test_sc_mc_coexistence_solves_equal_chemical_potentials():
    for G, total in ((1.5, 2.0), (1.2, 2.0), (3.0, 1.0)):
        a, b = studies.sc_mc_coexistence(G, total)
        assert abs(a + b - total) < 1e-12 and a > b > 0
        assert abs(math.log(a / b) - G * (a - b)) < 1e-9
    with pytest.raises(ValueError):
        studies.sc_mc_coexistence(0.9, 2.0)   # G_RB total / 2 <= 1: no demixing


def test_sc_mc_coexistence_against_the_oracle(orc):
    """A red slab in blue relaxed by the oracle (2-D, G_RB = 1.5, 8000 steps):
    the bulk pair it reaches, from the computed coexistence pair as from
    1.94 / 0.06, satisfies ln(a / b) = G (a - b) to 3 % (the lattice
    stencil's correction to the continuum relation); the computed pair,
    whose total (2) the interfaces shift, is within 5 % of its majority and
    20 % of its minority density (measured 1.950 / 0.117 against 1.859 /
    0.141)."""
    a, b = studies.sc_mc_coexistence(1.5, 2.0)
    x = np.arange(64)
    inside = np.abs(x - 31.5) < 16
    shape = (1, 4, 64)
    for maj, mino in ((a, b), (1.94, 0.06)):
        rR = np.broadcast_to(np.where(inside, maj, mino), shape).copy()
        rB = np.broadcast_to(np.where(inside, mino, maj), shape).copy()
        p = orc.make_params(lattice=0, model=2, nx=64, ny=4, nz=1, G_RB=1.5, rho0_R=2.0, rho0_B=2.0)
        f = orc.run(p, orc.init_equilibrium(p, rR, rB), 8000)
        r, bl, _ = orc.moments(p, f)
        A, B = r[0, 0, 32], bl[0, 0, 32]
        assert abs(math.log(A / B) - 1.5 * (A - B)) < 0.03 * math.log(A / B)
        assert abs(A - a) < 0.05 * a and abs(B - b) < 0.2 * b


def test_miller_scriven_reduces_to_lamb():
    sigma, R = 0.01, 20.0
    wl = studies.lamb_omega(sigma, R)
    assert abs(wl - math.sqrt(24 * sigma / (5 * R ** 3))) < 1e-15
    assert abs(studies.miller_scriven_omega(sigma, R, 1.0, 1.0, 1e-12, 1e-12) - wl) < 1e-6 * wl
    assert studies.miller_scriven_omega(sigma, R, 1.0, 1.0, 0.05, 0.05) < wl


def test_damped_cosine_fit_recovers_a_known_signal():
    t = 20.0 * np.arange(1, 1001)
    r = 21.0 + 1.5 * np.exp(-2e-4 * t) * np.cos(7e-4 * t + 0.4)
    w, lam, rd = studies.fit_damped_cosine(t, r, 6e-4)
    assert abs(w - 7e-4) < 1e-8 and abs(lam - 2e-4) < 1e-8 and abs(rd - 21.0) < 1e-8


def test_sc_pressure_equal_at_coexistence_and_flat_at_spinodals():
    """The equation of state the E_kin study uses for Young-Laplace gives
    equal pressures at the coexistence pair of the serving solver, and zero
    slope at the spinodals 1 + G x (1 - x) = 0, x = exp(-rho)."""
    from paper_2110_05197_amd import serve, sweeps
    for G in (-4.4, -5.0, -5.9):
        liq, gas = serve.sc_coexistence(G)
        assert abs(sweeps.sc_pressure(liq, G) - sweeps.sc_pressure(gas, G)) < 1e-12
        d = math.sqrt(1.0 + 4.0 / G)
        for x in ((1 + d) / 2, (1 - d) / 2):
            r, h = -math.log(x), 1e-6
            slope = (sweeps.sc_pressure(r + h, G) - sweeps.sc_pressure(r - h, G)) / (2 * h)
            assert abs(slope) < 1e-8


def test_contraction_sets_reproduce_printed_scales():
    """The contraction sets as transcribed give the capillary times and
    Ohnesorge numbers the contraction section prints for them: set 1
    t_cap = 262.9 and Oh = 0.1, sets 2-4 t_cap = 160 and Oh = 0.084."""
    sets = {c["name"]: c for c in studies.CONTR_SETS}
    c = sets["1"]
    tcap, u, Oh = studies.contraction_scales(c["rho"][0], c["sigma"], c["R0"], c["L"], c["tau"][0])
    assert abs(tcap - 262.9) < 0.05 and abs(Oh - 0.1) < 0.0005
    assert abs(u * tcap - c["R0"]) < 1e-9          # the end moves R0 per capillary time
    for name in ("2", "4"):
        c = sets[name]
        tcap, u, Oh = studies.contraction_scales(c["rho"][0], c["sigma"], c["R0"], c["L"], c["tau"][0])
        assert abs(tcap - 160.0) < 0.5 and abs(Oh - 0.084) < 0.0005


def test_laplace_measure_recovers_sigma_of_a_built_state():
    """sweeps.measure on observables built from a known droplet: interface
    radius R from the red volume, inside/outside densities whose pressure
    jump (Eq. CGpressure, colour sound speeds from Eq. gamma) is 2 sigma / R
    gives sigma_cal = sigma and E = |0.01 - sigma| / 0.01; E_kin per area
    uses the set radius when given."""
    from paper_2110_05197_amd import sweeps
    for gamma in (1.0, 37.4, 1000.0):
        p = dict(alpha_B=0.2, rho0_R=gamma, rho0_B=1.0)
        aR = 1.0 - 0.8 / gamma
        cR2, cB2 = (1.0 - aR) / 2.0, 0.4
        R, sigma, rho_out = 17.0, 0.0123, 1.01
        rho_in = (rho_out * cB2 + 2.0 * sigma / R) / cR2
        obs = dict(red_volume=4.0 / 3.0 * math.pi * R ** 3, mass_R=rho_in * 4.0 / 3.0 * math.pi * 15.0 ** 3,
                   rho_in=rho_in, rho_out=rho_out, ekin=2.5, eps_used=1 - 1e-10)
        m = sweeps.measure(obs, p, R0=16)
        assert abs(m["R"] - R) < 1e-12 and abs(m["R_equimolar"] - 15.0) < 1e-12
        assert abs(m["sigma_cal"] - sigma) < 1e-12
        assert abs(m["E"] - abs(0.01 - sigma) / 0.01) < 1e-10
        assert abs(m["ekin_per_area"] - 2.5 / (4.0 * math.pi * 256.0)) < 1e-15


def test_sc_laplace_pressure_jump_sign():
    """The SC equation of state gives a positive Young-Laplace jump for a
    liquid drop slightly above its coexistence density in slightly
    compressed vapour, and zero at the flat coexistence pair."""
    from paper_2110_05197_amd import serve, sweeps
    G = -5.0
    liq, gas = serve.sc_coexistence(G)
    assert abs(sweeps.sc_pressure(liq, G) - sweeps.sc_pressure(gas, G)) < 1e-12
    assert sweeps.sc_pressure(liq * 1.02, G) - sweeps.sc_pressure(gas, G) > 0
