"""Two-component Shan-Chen with the multirange forces (Eqs. benziforces,
doublebeltattractiveforce, doublebeltrepulsionforce, pweights) on the GPU:
parity with the oracle, batch invariance."""
import numpy as np
import pytest

from paper_2110_05197_amd import inputs

pytestmark = pytest.mark.gpu

# couplings of the droplet-collision study (Table dropcolParams, set 1), rho_0 = 0.83
BENZI = dict(G_RB=0.405, Ga_R=-9.0, Ga_B=-8.0, Gr_R=8.1, Gr_B=7.1, psi_rho0=0.83, rho0_X=0.83,
             rho0_R=1.18, rho0_B=0.18, tau_R=1.0, tau_B=0.8)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_05197_amd as M
    M.lib()
    return M


def fields(shape, seed):
    """Species A droplet (1.18 / 0.18 inside, swapped outside; total 1.36)
    with a little seeded noise and velocity."""
    frac, _ = inputs.droplet(shape, min(shape) / 3.0, 1.0, 1.0)
    rng = np.random.default_rng(seed)
    rA = 0.18 + frac + 0.01 * rng.standard_normal(shape)
    rB = 0.18 + (1.0 - frac) + 0.01 * rng.standard_normal(shape)
    u = 0.01 * rng.standard_normal((3,) + shape)
    return rA, rB, u


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5), (2, 2e-5)])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 2)])
def test_multirange_parity(M, orc, prec, tol, bc):
    shape = (16, 20, 24)
    rA, rB, u = fields(shape, 5)
    p = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=prec, nx=24, ny=20, nz=16, bc=bc, **BENZI)
    po = orc.make_params(**{k: p[k] for k in orc.DEFAULTS if k in p})
    fo = orc.run(po, orc.init_equilibrium(po, rA, rB, u), 100)
    s = M.Sim(p)
    assert s.kernel_used() == M.KERNEL_TWO_PASS
    s.init_equilibrium(rA, rB, u)
    st, done = s.step(100, check_every=100)
    assert st == M.OK and done == 100
    fg = s.export_f().cpu().numpy()
    e = float(np.abs(fg - fo).max() / np.abs(fo).max())
    og, oo = s.observables(), orc.observables(po, fo)
    say(f"[multirange] prec={prec} bc={bc}: rel max err {e:.2e} (tol {tol:g})")
    assert e <= tol
    for k in ("mass_R", "mass_B", "ekin"):
        assert og[k] == pytest.approx(oo[k], rel=max(tol * 10, 1e-12), abs=1e-14)
    s.close()


def test_multirange_batch_invariance(M):
    """A multirange simulation and a plain two-component one advanced in one
    batch each equal the same simulation stepped alone, bitwise (they run
    different collide kernels, so they must land in different groups)."""
    shape = (16, 20, 24)
    rA, rB, u = fields(shape, 8)
    pm = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=24, ny=20, nz=16,
                       kernel=M.KERNEL_TWO_PASS, **BENZI)
    pp = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=24, ny=20, nz=16,
                       G_RB=1.2, kernel=M.KERNEL_TWO_PASS)
    solo = M.Sim(pm)
    solo.init_equilibrium(rA, rB, u)
    solo.step(30)
    f_solo = solo.export_f().cpu().numpy()
    solo_p = M.Sim(pp)
    solo_p.init_equilibrium(rA + 0.3, rB + 0.3)
    solo_p.step(30)
    f_solo_p = solo_p.export_f().cpu().numpy()
    a, b = M.Sim(pm), M.Sim(pp)
    a.init_equilibrium(rA, rB, u)
    b.init_equilibrium(rA + 0.3, rB + 0.3)
    batch = M.Batch([a, b], [30, 30])
    for _ in range(3):
        batch.step(10, use_graph=True)
    st, steps = batch.status()
    batch.close()
    assert list(steps) == [30, 30]
    assert np.array_equal(a.export_f().cpu().numpy(), f_solo)
    assert np.array_equal(b.export_f().cpu().numpy(), f_solo_p)
    for s in (solo, solo_p, a, b):
        s.close()


@pytest.mark.parametrize("prec,bc", [(1, (0, 0, 0)), (0, (1, 1, 2)), (2, (0, 0, 0)), (3, (1, 1, 2))])
def test_multirange_staged_box_equals_field_reads(M, prec, bc):
    """The solo collide stages psi in LDS per 64 x 4 tile (and is compiled
    for a wave count of its own per precision); the batched one reads the
    field.  On a box of several tiles with ragged last tiles in x
    (130 = 64 + 64 + 2) and y (22 = 5 * 4 + 2) the two agree bitwise in every
    precision."""
    shape = (20, 22, 130)
    rA, rB, u = fields(shape, 11)
    p = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=prec, nx=130, ny=22, nz=20, bc=bc, **BENZI)
    solo = M.Sim(p)
    solo.init_equilibrium(rA, rB, u)
    solo.step(20)
    f_solo = solo.export_f().cpu().numpy()
    a = M.Sim(p)
    a.init_equilibrium(rA, rB, u)
    batch = M.Batch([a], [20])
    batch.step(20)
    batch.close()
    say(f"[multirange staged] prec={prec} bc={bc}: max |diff| "
        f"{float(np.abs(a.export_f().cpu().numpy() - f_solo).max()):.3e}")
    assert np.array_equal(a.export_f().cpu().numpy(), f_solo)
    for s in (solo, a):
        s.close()
