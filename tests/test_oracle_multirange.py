"""Pins of the oracle's two-component Shan-Chen multirange forces (Eqs.
benziforces, doublebeltattractiveforce, doublebeltrepulsionforce, pweights):
the neighbourhood and its weights, the forces on fields whose stencil sums
are known in closed form, pair antisymmetry, and conservation by the step."""
from fractions import Fraction
import math

import numpy as np
import pytest

BENZI = dict(G_RB=0.405, Ga_R=-9.0, Ga_B=-8.0, Gr_R=8.1, Gr_B=7.1, psi_rho0=0.83, rho0_X=0.83)


def test_belts_shells_and_isotropy(orc):
    """92 vectors in shells |c|^2 = 1,2,3,4,5,6,8 of 6,12,8,6,24,24,12;
    sum p c_x^2 = 1/3 (the gradient normalisation); isotropic moments to
    sixth order (c_x^4 : c_x^2 c_y^2 = 3, c_x^6 : c_x^4 c_y^2 : c_x^2 c_y^2 c_z^2
    = 15 : 3 : 1); belt 1 carries the D3Q19 weights, sum w c_x^2 = 1/3."""
    c, p, w = orc.belts_table()
    assert len(c) == 92 and len({tuple(v) for v in c}) == 92
    r2 = (c ** 2).sum(axis=1)
    assert sorted(np.unique(r2, return_counts=True)[1].tolist()) == sorted([6, 12, 8, 6, 24, 24, 12])
    frac = [Fraction(x).limit_denominator(20000) for x in p]
    cx, cy, cz = (c[:, d].tolist() for d in range(3))
    m = lambda ex, ey, ez: sum(f * (a ** ex) * (b ** ey) * (d ** ez) for f, a, b, d in zip(frac, cx, cy, cz))
    assert m(2, 0, 0) == Fraction(1, 3) == m(0, 2, 0) == m(0, 0, 2)
    assert m(1, 0, 0) == 0 and m(1, 1, 0) == 0 and m(3, 0, 0) == 0
    assert m(4, 0, 0) == 3 * m(2, 2, 0)
    assert m(6, 0, 0) == 15 * m(2, 2, 2) and m(4, 2, 0) == 3 * m(2, 2, 2)
    belt1 = r2 <= 2
    assert np.all(w[~belt1] == 0) and np.isclose((w * c[:, 0] ** 2).sum(), 1 / 3, rtol=0, atol=1e-15)
    assert np.allclose(w[r2 == 1], 1 / 18) and np.allclose(w[r2 == 2], 1 / 36)


def _psi_inverse(psi, rho0):
    return -rho0 * np.log(1.0 - psi / rho0)


@pytest.mark.parametrize("coef", [(0.01, 0.0), (0.01, 0.0004)])
def test_forces_on_a_quadratic_pseudopotential(orc, coef):
    """psi_R(x) = 0.2 + a x + b x^2 (rho_R chosen to give it), rho_B uniform,
    walls on x: at interior nodes (2 from the faces) the belt sums are exact
    derivatives, so F_R = -(G^a_R + G^r_R) psi_R(x) psi_R'(x) / 3 x-hat and
    F_B = -(G_RB / rho_0^2) rho_B grad(rho_R) / 3 (cross term, belt 1)."""
    a, b = coef
    nx, ny, nz = 16, 6, 6
    x = np.arange(nx, dtype=float)
    psi = 0.2 + a * x + b * x * x
    rho0 = BENZI["psi_rho0"]
    rR = np.broadcast_to(_psi_inverse(psi, rho0), (nz, ny, nx)).copy()
    rB = np.full((nz, ny, nx), 0.3)
    p = orc.make_params(lattice=1, model=2, nx=nx, ny=ny, nz=nz, bc=(1, 0, 0), **BENZI)
    f = orc.init_equilibrium(p, rR, rB)
    FR, FB = orc.sc_forces(p, f)
    xi = np.arange(2, nx - 2)
    dpsi = a + 2 * b * x[xi]
    expect_R = -(BENZI["Ga_R"] + BENZI["Gr_R"]) * psi[xi] * dpsi / 3
    # the cross force on red vanishes (rho_B uniform); on blue it follows
    # the belt-1 gradient of rho_R, exact only where rho_R is locally
    # quadratic, so it is checked for sign and direction only
    assert np.allclose(FR[0, 3, 3, xi], expect_R, rtol=1e-9, atol=1e-14)
    assert np.allclose(FR[1:], 0, atol=1e-14) and np.allclose(FB[1:], 0, atol=1e-14)
    assert np.all(FB[0, 3, 3, xi] * np.sign(np.gradient(rR[3, 3])[xi]) < 0)


def test_forces_pairwise_antisymmetric(orc):
    """On a periodic box every pair interaction appears with both signs, so
    the total of each force over the lattice vanishes."""
    rng = np.random.default_rng(4)
    shape = (10, 9, 12)
    rR = rng.uniform(0.1, 1.2, shape)
    rB = rng.uniform(0.1, 1.2, shape)
    p = orc.make_params(lattice=1, model=2, nx=12, ny=9, nz=10, **BENZI)
    FR, FB = orc.sc_forces(p, orc.init_equilibrium(p, rR, rB))
    tot = (FR + FB).reshape(3, -1).sum(axis=1)
    scale = np.abs(FR).sum()
    assert np.all(np.abs(tot) < 1e-13 * scale)
    # each species' multirange self-force alone also sums to zero
    p0 = dict(p, G_RB=0.0)
    FR0, FB0 = orc.sc_forces(p0, orc.init_equilibrium(p0, rR, rB))
    assert np.all(np.abs(FR0.reshape(3, -1).sum(axis=1)) < 1e-13 * np.abs(FR0).sum())
    assert np.all(np.abs(FB0.reshape(3, -1).sum(axis=1)) < 1e-13 * np.abs(FB0).sum())


def test_multirange_reaches_two_nodes(orc):
    """A single perturbed node moves the force two nodes away along an axis
    (belt 2) but not three."""
    shape = (9, 9, 9)
    rR = np.full(shape, 0.5)
    rR[4, 4, 4] = 0.7
    rB = np.full(shape, 0.5)
    p = orc.make_params(lattice=1, model=2, nx=9, ny=9, nz=9, **dict(BENZI, G_RB=0.0))
    FR, _ = orc.sc_forces(p, orc.init_equilibrium(p, rR, rB))
    F0, _ = orc.sc_forces(p, orc.init_equilibrium(p, np.full(shape, 0.5), rB))
    dF = FR - F0
    assert abs(dF[0, 4, 4, 6]) > 1e-6 and abs(dF[0, 4, 4, 2]) > 1e-6
    assert dF[0, 4, 4, 7] == 0 and dF[0, 4, 4, 1] == 0 and dF[0, 4, 7, 4] == 0


def test_multirange_step_conserves_mass_and_momentum(orc):
    rng = np.random.default_rng(9)
    shape = (8, 10, 12)
    rR = 0.18 + rng.uniform(0, 1.0, shape)
    rB = 1.36 - rR
    p = orc.make_params(lattice=1, model=2, nx=12, ny=10, nz=8, tau_R=1.0, tau_B=1.0, **BENZI)
    f = orc.init_equilibrium(p, rR, rB)
    o0 = orc.observables(p, f)
    f = orc.run(p, f, 40)
    o1 = orc.observables(p, f)
    assert abs(o1["mass_R"] - o0["mass_R"]) < 1e-12 * o0["mass_R"]
    assert abs(o1["mass_B"] - o0["mass_B"]) < 1e-12 * o0["mass_B"]
    # momentum (with the half-force term) stays at its initial value
    for k in ("mom_x", "mom_y", "mom_z"):
        if k in o0:
            assert abs(o1[k] - o0[k]) < 1e-11
    assert o1["diverged"] == 0
