"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element.

Tolerances: relative max-norm error max|f_gpu - f_oracle| / max|f_oracle|
(and the same on rho_k) <= 1e-10 for the FP64 path and <= 2e-5 for FP32
after 100 steps.  FP16 storage and the mixed path report their error.
"""
import sys

import numpy as np
import pytest

from paper_2110_05197_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_05197_amd as M
    M.lib()
    return M


def torch_sync():
    import torch
    torch.cuda.synchronize()


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_run(M, p, rR, rB, u, steps, kernel=None):
    q = dict(p)
    if kernel is not None:
        q["kernel"] = kernel
    sim = M.Sim(q)
    sim.init_equilibrium(rR, rB, u)
    st, done = sim.step(steps, check_every=steps if steps else 0)
    assert st == M.OK and done == steps
    f = sim.export_f().cpu().numpy()
    return sim, f


def compare(M, orc, p, rR, rB, u, steps, tol, kernel=None, label=""):
    say(f"[parity] {label} shape={(p['nz'], p['ny'], p['nx'])} lattice={p['lattice']} "
        f"model={p['model']} prec={p['precision']} kernel={kernel} steps={steps}")
    fo = orc.run(p, orc.init_equilibrium(p, rR, rB, u), steps)
    sim, fg = gpu_run(M, p, rR, rB, u, steps, kernel)
    e_f = rel_err(fg, fo)
    ro = fo.sum(axis=1)
    rg = fg.sum(axis=1)
    e_r = rel_err(rg, ro)
    say(f"    rel max err f={e_f:.3e} rho={e_r:.3e} (tol {tol:g})")
    assert e_f <= tol and e_r <= tol
    return sim, fg, fo


def cg_droplet_case(shape, seed, gamma=1.0, lattice=1, **kw):
    rho0_B = 1.0 / gamma
    R = min(s for s in shape if s > 1) / 4.0
    rR, rB = inputs.droplet(shape, R, 1.0, rho0_B)
    rR = rR * (1 + inputs.noise(shape, 0.01, seed))
    rB = rB * (1 + inputs.noise(shape, 0.01, seed + 1))
    u = np.zeros((3,) + shape)
    for a in range(2 if lattice == 0 else 3):
        u[a] = inputs.noise(shape, 0.02, seed + 2 + a)
    return rR, rB, u


# --------------------------------------------------------------------------
# Colour gradient
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", [1, 2])
def test_cg_d2q9_fp64_static_droplet(M, orc, kernel):
    """64x64 D2Q9 droplet R = 16, A = 0.01, tau = 1, beta = 0.7, FP64."""
    p = M.make_params(lattice=M.D2Q9, model=M.CG, precision=M.FP64, nx=64, ny=64, nz=1, A=0.01)
    rR, rB = inputs.droplet((1, 64, 64), 16.0)
    compare(M, orc, p, rR, rB, None, 100, 1e-10, kernel=kernel, label="cg-d2q9-config1")


@pytest.mark.parametrize("kernel", [1, 2])
def test_cg_d2q9_fp64_ragged_moving(M, orc, kernel):
    shape = (1, 45, 70)
    p = M.make_params(lattice=M.D2Q9, precision=M.FP64, nx=70, ny=45, nz=1, A=0.03, tau_R=0.7,
                      tau_B=1.2, rho0_B=0.1)
    rR, rB, u = cg_droplet_case(shape, 11, gamma=10.0, lattice=0)
    compare(M, orc, p, rR, rB, u, 100, 1e-10, kernel=kernel, label="cg-d2q9-ragged")


def test_cg_d3q19_fp64_ragged_density_ratio(M, orc):
    shape = (30, 36, 40)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP64, nx=40, ny=36, nz=30, A=0.02, tau_R=0.7,
                      tau_B=1.1, rho0_B=0.1)
    rR, rB, u = cg_droplet_case(shape, 12, gamma=10.0)
    compare(M, orc, p, rR, rB, u, 100, 1e-10, label="cg-d3q19-fp64")


def test_cg_d3q19_fp64_plain_equilibrium(M, orc):
    shape = (16, 20, 24)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP64, nx=24, ny=20, nz=16, A=0.02,
                      enhanced_eq=0, rho0_B=0.5)
    rR, rB, u = cg_droplet_case(shape, 13, gamma=2.0)
    compare(M, orc, p, rR, rB, u, 100, 1e-10, label="cg-d3q19-plain-eq")


@pytest.mark.parametrize("kernel", [1, 2])
def test_cg_d3q19_fp32(M, orc, kernel):
    shape = (24, 32, 64)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=64, ny=32, nz=24, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 14)
    compare(M, orc, p, rR, rB, u, 100, 2e-5, kernel=kernel, label="cg-d3q19-fp32")


@pytest.mark.parametrize("kernel", [1, 2])
def test_cg_d3q19_fp32_density_ratio_tile_shapes(M, orc, kernel):
    # nx = 80: a 64-wide column and a masked 16-wide edge column; ny = 20: 4-row tiles
    shape = (18, 20, 80)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=80, ny=20, nz=18, A=0.02,
                      rho0_B=0.1, tau_R=0.8, tau_B=1.0)
    rR, rB, u = cg_droplet_case(shape, 15, gamma=10.0)
    compare(M, orc, p, rR, rB, u, 100, 2e-5, kernel=kernel, label="cg-d3q19-fp32-gamma10")


@pytest.mark.parametrize("prec,tol", [(3, 5e-3), (2, 2e-5)])
def test_cg_d3q19_fp16_and_mixed_error(M, orc, prec, tol):
    shape = (16, 16, 32)
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=32, ny=16, nz=16, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 16)
    compare(M, orc, p, rR, rB, u, 100, tol, label=f"cg-d3q19-prec{prec}")


def test_mixed_beats_fp32_at_density_ratio_1000(M, orc):
    """gamma = 1000 (rho_R^0 = 1000, rho_B^0 = 1, so that the ambient pressure
    rho_B c_sB^2 = 0.4 dwarfs the Laplace pressure): the mixed path's error
    against the oracle in the light phase's density is no worse than plain
    FP32 shifted storage, and both stay within the FP32 tolerance."""
    shape = (16, 16, 32)
    res = {}
    for prec in (1, 2):
        p = M.make_params(lattice=M.D3Q19, precision=prec, nx=32, ny=16, nz=16, A=0.01,
                          rho0_R=1000.0, rho0_B=1.0, tau_R=1.0, tau_B=0.55)
        rR, rB = inputs.ligament(shape, 4.0, 20.0, 1000.0, 1.0, axis=0)
        say(f"[parity] gamma=1000 prec={prec}")
        fo = orc.run(p, orc.init_equilibrium(p, rR, rB, None), 100)
        assert orc.observables(p, fo)["diverged"] == 0
        _, fg = gpu_run(M, p, rR, rB, None, 100)
        eB = float(np.abs(fg[1].sum(axis=0) - fo[1].sum(axis=0)).max())
        res[prec] = (rel_err(fg, fo), eB)
        say(f"    prec={prec} rel err f={res[prec][0]:.3e} light-phase rho abs err={eB:.3e}")
    assert res[1][0] <= 2e-5 and res[2][0] <= 2e-5
    assert res[2][1] <= res[1][1] * 1.01


# --------------------------------------------------------------------------
# The one-pass kernel as the benchmark runs it: every block marches many
# planes (the plane-(z+2) prefetch, the four-plane LDS ring and the rotation
# through the per-thread slot all execute), 100 steps against the oracle.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec,bc,tol,min_planes", [(1, (0, 0, 0), 2e-5, 8), (0, (0, 0, 0), 1e-10, 16),
                                                    (1, (1, 1, 2), 2e-5, 8), (0, (1, 1, 2), 1e-10, 16),
                                                    (2, (0, 0, 0), 2e-5, 8)])
def test_cg_d3q19_deep_march(M, orc, prec, bc, tol, min_planes):
    """256 x 64 x 64, density ratio 10, droplet with 1 % density and 0.02
    velocity noise: 4 x 8 columns of 64 x 8 (64 x 4 in FP64), so each block
    marches 8 (16) planes."""
    shape = (64, 64, 256)
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=256, ny=64, nz=64, bc=bc, A=0.02,
                      rho0_B=0.1, tau_R=0.8, tau_B=1.0)
    rR, rB, u = cg_droplet_case(shape, 41, gamma=10.0)
    if bc[2] == 2:
        u[2] += 0.01
    sim = M.Sim(dict(p, kernel=2))
    tx, ty, planes = sim.fused_tile()
    say(f"[deep march] prec={prec} bc={bc}: {tx}x{ty} columns, {planes} planes per block")
    assert planes >= min_planes
    compare(M, orc, p, rR, rB, u, 100, tol, kernel=2, label="cg-d3q19-deep-march")


def test_cg_d2q9_fp32_row_kernel(M, orc):
    """D2Q9 FP32 at 1024 x 512 = 2^19 nodes, where the automatic choice is
    the one-pass row kernel (rows of 256 marching along y), 100 steps."""
    shape = (1, 512, 1024)
    p = M.make_params(lattice=M.D2Q9, precision=M.FP32, nx=1024, ny=512, nz=1, A=0.02, rho0_B=0.5,
                      tau_R=0.7, tau_B=1.0)
    rR, rB, u = cg_droplet_case(shape, 42, gamma=2.0, lattice=0)
    sim = M.Sim(p)
    assert sim.kernel_used() == M.KERNEL_FUSED
    tx, ty, rows = sim.fused_tile()
    say(f"[d2q9 row kernel] {tx}-node row segments, {rows} rows per block")
    assert rows >= 8
    compare(M, orc, p, rR, rB, u, 100, 2e-5, label="cg-d2q9-fp32-row-kernel")


@pytest.mark.parametrize("prec", [1, 0, 2, 3])
def test_deep_march_fused_equals_two_pass_bitwise(M, prec):
    """The one-pass kernel with 8-16 planes per block equals the two-pass
    kernels bit for bit (colour gradient, periodic and walls + outflow)."""
    shape = (64, 64, 256)
    for bc in ((0, 0, 0), (1, 1, 2)):
        p = M.make_params(lattice=M.D3Q19, precision=prec, nx=256, ny=64, nz=64, bc=bc, A=0.02,
                          rho0_B=0.1, tau_R=0.8, tau_B=1.0)
        rR, rB, u = cg_droplet_case(shape, 43, gamma=10.0)
        say(f"[bitwise deep march] prec={prec} bc={bc}")
        s1, f1 = gpu_run(M, p, rR, rB, u, 29, kernel=1)
        s2, f2 = gpu_run(M, p, rR, rB, u, 29, kernel=2)
        assert s2.fused_tile()[2] >= 8
        assert np.array_equal(f1, f2)


@pytest.mark.parametrize("prec,bc,tol", [(1, (0, 0, 0), 2e-5), (2, (1, 1, 2), 2e-5)])
def test_cg_96_wide_columns(M, orc, prec, bc, tol):
    """nx = 96 (96 divides it, 64 does not): one column of 96 x 4 per row
    band instead of a 64-wide column and a half-idle masked one; 96 x 96 x 80,
    24 columns x 10 z-chunks of 8 planes, 100 steps against the oracle."""
    shape = (80, 96, 96)
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=96, ny=96, nz=80, bc=bc, A=0.02,
                      rho0_B=0.1, tau_R=0.8, tau_B=1.0)
    rR, rB, u = cg_droplet_case(shape, 44, gamma=10.0)
    sim = M.Sim(p)
    assert sim.kernel_used() == M.KERNEL_FUSED
    tx, ty, planes = sim.fused_tile()
    say(f"[96-wide] prec={prec} bc={bc}: {tx}x{ty} columns, {planes} planes per block")
    assert (tx, ty) == (96, 4) and planes >= 8
    sim.close()
    compare(M, orc, p, rR, rB, u, 100, tol, label="cg-96-wide")


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("model", ["CG", "SC_MP", "SC_MC"])
def test_96_wide_columns_equal_two_pass_bitwise(M, prec, model):
    """The 96 x 4 columns of the one-pass kernel equal the two-pass kernels
    bit for bit, every model, periodic and walls + outflow (and, for the
    colour gradient in FP32 and mixed, with conserve_mass)."""
    shape = (40, 96, 96)
    for bc in ((0, 0, 0), (1, 1, 2)):
        if model == "SC_MP":
            p = M.make_params(lattice=M.D3Q19, model=M.SC_MP, precision=prec, nx=96, ny=96, nz=40, bc=bc,
                              G=-5.0, rho0_R=1.9, rho0_B=0.12)
            a, b = inputs.droplet(shape, 20.0, 1.9, 0.12)
            rR, rB, u = a + b, None, None
        elif model == "SC_MC":
            p = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=prec, nx=96, ny=96, nz=40, bc=bc,
                              G_RB=1.2)
            rR, rB, u = cg_droplet_case(shape, 45, gamma=1.0)
        else:
            p = M.make_params(lattice=M.D3Q19, precision=prec, nx=96, ny=96, nz=40, bc=bc, A=0.02,
                              rho0_B=0.1, tau_R=0.8, tau_B=1.0)
            rR, rB, u = cg_droplet_case(shape, 46, gamma=10.0)
        cons = (0, 1) if model == "CG" and prec in (1, 2) else (0,)
        for c in cons:
            q = dict(p, conserve_mass=c)
            say(f"[bitwise 96-wide] model={model} prec={prec} bc={bc} conserve_mass={c}")
            s1, f1 = gpu_run(M, q, rR, rB, u, 17, kernel=1)
            s2, f2 = gpu_run(M, q, rR, rB, u, 17, kernel=2)
            assert s2.fused_tile()[:2] == (96, 4) and s2.fused_tile()[2] >= 4
            assert np.array_equal(f1, f2)
            s1.close()
            s2.close()


# --------------------------------------------------------------------------
# Boundaries (walls on x/y, outflow on z)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec,kernel,tol", [(0, 1, 1e-10), (0, 2, 1e-10), (1, 1, 2e-5), (1, 2, 2e-5)])
def test_cg_walls_outflow(M, orc, prec, kernel, tol):
    shape = (40, 16, 32)
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=32, ny=16, nz=40, bc=(1, 1, 2),
                      A=0.02, rho0_B=0.1, tau_R=1.0, tau_B=0.6)
    rR, rB = inputs.ligament(shape, 5.0, 30.0, 1.0, 0.1, axis=2)
    u = np.zeros((3,) + shape)
    u[2] = 0.01
    compare(M, orc, p, rR, rB, u, 100, tol, kernel=kernel, label="cg-walls-outflow")


@pytest.mark.parametrize("kernel", [1, 2])
def test_cg_d2q9_walls(M, orc, kernel):
    shape = (1, 30, 50)
    p = M.make_params(lattice=M.D2Q9, precision=M.FP64, nx=50, ny=30, nz=1, bc=(2, 1, 0), A=0.02)
    rR, rB, u = cg_droplet_case(shape, 17, lattice=0)
    compare(M, orc, p, rR, rB, u, 100, 1e-10, kernel=kernel, label="cg-d2q9-walls")


# --------------------------------------------------------------------------
# Shan-Chen variants and the repulsion force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,prec,kernel,tol", [(1, 0, 1, 1e-10), (1, 1, 1, 2e-5), (1, 1, 2, 2e-5),
                                                     (1, 0, 2, 1e-10), (0, 0, 1, 1e-10), (0, 0, 2, 1e-10),
                                                     (0, 1, 2, 2e-5)])
def test_sc_multiphase(M, orc, lattice, prec, kernel, tol):
    shape = (16, 16, 32) if lattice == 1 else (1, 40, 48)
    p = M.make_params(lattice=lattice, model=M.SC_MP, precision=prec, nx=shape[2], ny=shape[1],
                      nz=shape[0], G=-5.0, tau_R=0.9, rho0_R=1.9, rho0_B=0.12)
    rR, rB = inputs.droplet(shape, 6.0, 1.9, 0.12)
    rho = rR + rB + inputs.noise(shape, 0.01, 18)
    compare(M, orc, p, rho, None, None, 100, tol, kernel=kernel, label="sc-mp")


@pytest.mark.parametrize("lattice,prec,kernel,tol", [(1, 0, 1, 1e-10), (1, 1, 2, 2e-5), (1, 0, 2, 1e-10),
                                                     (0, 0, 1, 1e-10), (0, 0, 2, 1e-10), (0, 1, 2, 2e-5)])
def test_sc_two_component(M, orc, lattice, prec, kernel, tol):
    shape = (16, 16, 32) if lattice == 1 else (1, 40, 48)
    p = M.make_params(lattice=lattice, model=M.SC_MC, precision=prec, nx=shape[2], ny=shape[1],
                      nz=shape[0], G_RB=1.2, tau_R=1.0, tau_B=0.8, rho0_R=1.0, rho0_B=1.0)
    rR, rB = inputs.droplet(shape, 6.0, 1.0, 1.0)
    compare(M, orc, p, rR + 0.04, rB + 0.04, None, 100, tol, kernel=kernel, label="sc-mc")


@pytest.mark.parametrize("lattice", [0, 1])
def test_cg_repulsion(M, orc, lattice):
    shape = (1, 32, 48) if lattice == 0 else (12, 16, 32)
    nx = shape[2]
    x = np.arange(nx, dtype=float)
    films = (nx / 4 - 0.5, 3 * nx / 4 - 0.5)
    dist = np.min([np.abs(x - c - nx * np.round((x - c) / nx)) for c in films], axis=0)
    phi = np.broadcast_to(np.tanh((dist - 2.5) / 2.0), shape)
    rR = 0.5 * (1 + phi) * (1 + inputs.noise(shape, 0.01, 19))
    rB = 0.5 * (1 - phi)
    p = M.make_params(lattice=lattice, precision=M.FP64, nx=nx, ny=shape[1], nz=shape[0],
                      A=0.02, Pi=0.01, chi=1.0)
    compare(M, orc, p, rR, rB, None, 100, 1e-10, label="cg-repulsion")


# --------------------------------------------------------------------------
# Moments, observables, invariants of the GPU path itself
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model", [0, 1, 2])
def test_moments_and_observables_fp64(M, orc, model):
    shape = (12, 16, 20)
    kw = dict(G=-5.0, rho0_R=1.9, rho0_B=0.12) if model == 1 else dict(G_RB=1.2, A=0.02)
    p = M.make_params(lattice=M.D3Q19, model=model, precision=M.FP64, nx=20, ny=16, nz=12, **kw)
    if model == 1:
        rR, rB = inputs.droplet(shape, 4.0, 1.9, 0.12)
        rR, rB = rR + rB, None
    else:
        rR, rB = inputs.droplet(shape, 4.0)
        rR, rB = rR + 0.02, rB + 0.02
    say(f"[parity] moments/observables model={model}")
    fo = orc.run(p, orc.init_equilibrium(p, rR, rB, None), 30)
    sim, fg = gpu_run(M, p, rR, rB, None, 30)
    oo = orc.observables(p, fo)
    og = sim.observables()
    for k in ("mass_R", "mass_B", "mom_x", "mom_y", "mom_z", "ekin", "umax", "rho_in", "rho_out",
              "red_volume", "n_in", "n_out", "eps_used", "diverged"):
        scale = max(abs(oo[k]), 1e-300)
        if k.startswith("mom"):
            scale = max(scale, oo["mass_R"])
        assert abs(og[k] - oo[k]) <= 1e-10 * scale, (k, og[k], oo[k])
    rRg, rBg, ug = [t.cpu().numpy() for t in sim.moments()]
    rRo, rBo, jo = orc.moments(p, fo)
    assert rel_err(rRg, rRo) < 1e-12
    if model != 1:
        assert rel_err(rBg, rBo) < 1e-12
    if model == 0:   # bare velocity for CG
        uo = jo / (rRo + rBo)
        assert np.abs(ug - uo).max() < 1e-12


def test_fp32_mass_conservation(M):
    shape = (32, 32, 64)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=64, ny=32, nz=32, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 20)
    sim = M.Sim(p)
    sim.init_equilibrium(rR, rB, u)
    o0 = sim.observables()
    sim.step(500)
    o1 = sim.observables()
    say(f"[fp32 mass] drift R {abs(o1['mass_R'] - o0['mass_R']) / o0['mass_R']:.2e} "
        f"B {abs(o1['mass_B'] - o0['mass_B']) / o0['mass_B']:.2e}")
    # FP32 rounding at interface nodes: about 1e-7 of the colour mass per step
    assert abs(o1["mass_R"] - o0["mass_R"]) / o0["mass_R"] < 500 * 2e-7
    assert abs(o1["mass_B"] - o0["mass_B"]) / o0["mass_B"] < 500 * 2e-7


@pytest.mark.parametrize("prec", [1, 2])
def test_conserve_mass_option(M, orc, prec):
    """conserve_mass = 1 (FP32 and mixed storage): the rest population is set
    from FP64 sums so that each colour's node mass is kept to one rounding.
    The populations stay within the precision's bound of the FP64 oracle after
    100 steps, one-pass, two-pass and batched kernels still agree bit for bit
    (periodic, walls + outflow, and the D2Q9 row kernel),
    and the colour masses drift far less over 500 steps.  What remains is the
    single rounding of each node's rest population, whose errors do not quite
    cancel (about 3 % of an ulp per interface node and step).  Measured on this
    state: FP32 5.5e-7 against 7.5e-5 without (bound: 2e-9 per step and 20x
    less); mixed precision, whose sums and recolouring are FP64 already,
    2.1e-6 against 4.1e-6 (bound: 1e-8 per step and no more than without)."""
    shape = (24, 16, 64)
    p = M.make_params(lattice=M.D3Q19, precision=prec, nx=64, ny=16, nz=24, A=0.02, conserve_mass=1)
    rR, rB, u = cg_droplet_case(shape, 21)
    compare(M, orc, p, rR, rB, u, 100, 2e-5, kernel=2, label=f"conserve-mass prec={prec}")
    _, f_fused = gpu_run(M, p, rR, rB, u, 40, kernel=2)
    _, f_two = gpu_run(M, p, rR, rB, u, 40, kernel=1)
    assert np.array_equal(f_fused, f_two)
    sims = []
    for q in (p, dict(p, conserve_mass=0)):
        s = M.Sim(q)
        s.init_equilibrium(rR, rB, u)
        sims.append(s)
    b = M.Batch(sims, [40, 40])
    for _ in range(4):
        b.step(10)
    b.close()
    assert np.array_equal(sims[0].export_f().cpu().numpy(), f_fused)
    _, f_plain = gpu_run(M, dict(p, conserve_mass=0), rR, rB, u, 40, kernel=2)
    assert np.array_equal(sims[1].export_f().cpu().numpy(), f_plain)
    assert not np.array_equal(f_plain, f_fused)
    for s in sims:
        s.close()
    # the other conserving one-pass kernels: walls + outflow, and the D2Q9 rows
    for q, shape2, seed in ((dict(p, bc=(1, 1, 2)), shape, 22),
                            (M.make_params(lattice=M.D2Q9, precision=prec, nx=80, ny=48, nz=1, A=0.02,
                                           conserve_mass=1), (1, 48, 80), 23)):
        r2, b2, u2 = cg_droplet_case(shape2, seed, lattice=q["lattice"])
        _, g1 = gpu_run(M, q, r2, b2, u2, 30, kernel=2)
        _, g2 = gpu_run(M, q, r2, b2, u2, 30, kernel=1)
        assert np.array_equal(g1, g2), q["lattice"]
    drift = {}
    for c in (1, 0):
        sim = M.Sim(dict(p, conserve_mass=c))
        sim.init_equilibrium(rR, rB, u)
        o0 = sim.observables()
        sim.step(500)
        o1 = sim.observables()
        drift[c] = max(abs(o1[k] - o0[k]) / o0[k] for k in ("mass_R", "mass_B"))
        sim.close()
    say(f"[conserve_mass] prec={prec}: 500-step colour-mass change {drift[1]:.2e} (off: {drift[0]:.2e})")
    if prec == M.FP32:
        assert drift[1] < 500 * 2e-9 and drift[1] < drift[0] / 20
    else:
        assert drift[1] < 500 * 1e-8 and drift[1] <= drift[0]


@pytest.mark.parametrize("prec", [1, 0, 2, 3])
def test_fused_equals_two_pass_bitwise(M, prec):
    """The one-pass kernel and the two-pass kernels give bitwise identical
    populations (same node arithmetic), for every precision path, periodic
    and walls + outflow, all three models, 64-wide columns only and with a
    masked last column (nx = 88: 64 + 24; nx = 40: one masked column)."""
    for shape, bc in (((20, 16, 64), (0, 0, 0)), ((20, 16, 64), (1, 1, 2)), ((12, 8, 88), (0, 0, 0)),
                      ((12, 8, 40), (1, 0, 2))):
        for model in (0, 1, 2):
            kw = dict(G=-5.0, rho0_R=1.9, rho0_B=0.12) if model == 1 else dict(G_RB=1.2, A=0.02)
            p = M.make_params(lattice=M.D3Q19, model=model, precision=prec, nx=shape[2], ny=shape[1],
                              nz=shape[0], bc=bc, **kw)
            if model == 1:
                a, b = inputs.droplet(shape, 5.0, 1.9, 0.12)
                rR, rB = a + b, None
            else:
                rR, rB, _ = cg_droplet_case(shape, 21)
            say(f"[bitwise] fused vs two-pass prec={prec} shape={shape} bc={bc} model={model}")
            _, f1 = gpu_run(M, p, rR, rB, None, 37, kernel=1)
            _, f2 = gpu_run(M, p, rR, rB, None, 37, kernel=2)
            assert np.array_equal(f1, f2)


@pytest.mark.parametrize("prec", [1, 0, 2, 3])
def test_fused_equals_two_pass_bitwise_d2q9(M, prec):
    """D2Q9 one-pass kernel (rows of 256 marching along y; the box seen as
    nx x 1 x ny) against the two-pass kernels, bitwise: every precision, all
    three models, periodic, walls + outflow, full and masked row segments."""
    for shape, bc in (((1, 40, 512), (0, 0, 0)), ((1, 33, 300), (0, 0, 0)), ((1, 48, 300), (1, 2, 0)),
                      ((1, 20, 64), (2, 1, 0))):
        for model in (0, 1, 2):
            kw = dict(G=-5.0, rho0_R=1.9, rho0_B=0.12) if model == 1 else dict(G_RB=1.2, A=0.02)
            p = M.make_params(lattice=M.D2Q9, model=model, precision=prec, nx=shape[2], ny=shape[1], nz=1,
                              bc=bc, **kw)
            if model == 1:
                a, b = inputs.droplet(shape, 6.0, 1.9, 0.12)
                rR, rB = a + b, None
            else:
                rR, rB, _ = cg_droplet_case(shape, 27, lattice=0)
            say(f"[bitwise d2q9] fused vs two-pass prec={prec} shape={shape} bc={bc} model={model}")
            _, f1 = gpu_run(M, p, rR, rB, None, 41, kernel=1)
            _, f2 = gpu_run(M, p, rR, rB, None, 41, kernel=2)
            assert np.array_equal(f1, f2)


@pytest.mark.parametrize("lattice,shape,bc", [
    (1, (2, 4, 2), (0, 0, 0)), (1, (2, 4, 3), (1, 0, 2)), (1, (3, 8, 65), (0, 1, 0)),
    (1, (5, 4, 130), (2, 0, 1)), (0, (1, 2, 2), (0, 0, 0)), (0, (1, 3, 257), (1, 2, 0)),
    (0, (1, 1000, 3), (0, 0, 0)), (0, (1, 9, 513), (2, 1, 0))])
def test_fused_degenerate_boxes(M, orc, lattice, shape, bc):
    """Boxes of two or three nodes along an axis (halos that wrap onto the
    column itself, a single masked column or row segment), long thin boxes
    and a one-node edge segment: the one-pass kernel equals the two-pass
    kernels bit for bit (FP32) and the FP64 oracle to 1e-10 (FP64)."""
    nz, ny, nx = shape
    say(f"[degenerate] lattice={lattice} shape={shape} bc={bc}")
    for prec in (1, 0):
        p = M.make_params(lattice=lattice, precision=prec, nx=nx, ny=ny, nz=nz, bc=bc, A=0.02)
        rR, rB, u = cg_droplet_case(shape, 31, lattice=lattice)
        if prec == 1:
            _, f1 = gpu_run(M, p, rR, rB, u, 23, kernel=1)
            _, f2 = gpu_run(M, p, rR, rB, u, 23, kernel=2)
            assert np.array_equal(f1, f2)
        else:
            compare(M, orc, p, rR, rB, u, 23, 1e-10, kernel=2, label="degenerate")


def test_checkpoint_restore_bitwise(M):
    shape = (16, 16, 32)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=32, ny=16, nz=16, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 22)
    a = M.Sim(p)
    a.init_equilibrium(rR, rB, u)
    a.step(40)
    buf, st = a.checkpoint()
    a.step(40)
    fa = a.export_f().cpu().numpy()
    b = M.Sim(p)
    b.init_equilibrium(rR, rB, u)
    b.restore(buf, st)
    b.step(40)
    assert b.observables()["step"] == 80
    assert np.array_equal(b.export_f().cpu().numpy(), fa)


def test_divergence_is_detected(M):
    shape = (8, 8, 32)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=32, ny=8, nz=8, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 23)
    s = M.Sim(p)
    s.init_equilibrium(rR, rB, u)
    f = s.export_f()
    f[0, 3, 2, 2, 2] = float("nan")
    s.import_f(f)
    assert s.diverged()           # the check scans the current state itself
    s.import_f(f)
    st, done = s.step(50, check_every=10)
    assert st == M.DIVERGED and done == 10
    assert s.observables()["diverged"] == 1.0


def test_batch_reports_a_bad_final_state(M):
    """A sim whose last state is bad (here: imported with a NaN and given no
    steps to take) is reported STOPPED_DIVERGED by the batch status, not
    DONE, while a healthy one is DONE; a sim that diverges while stepping
    stops early."""
    shape = (8, 8, 64)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=64, ny=8, nz=8, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 25)
    sims = []
    for bad in (True, False, True):
        s = M.Sim(p)
        s.init_equilibrium(rR, rB, u)
        if bad:
            f = s.export_f()
            f[1, 5, 3, 3, 3] = float("nan")
            s.import_f(f)
        sims.append(s)
    b = M.Batch(sims, [0, 12, 12])
    b.step(4, use_graph=False)
    st, steps = b.status()
    assert st[0] == M.STOPPED_DIVERGED and steps[0] == 0
    assert st[2] == M.STOPPED_DIVERGED and steps[2] < 12
    b.step(10, use_graph=False)
    st, steps = b.status()
    assert st == [M.STOPPED_DIVERGED, M.DONE, M.STOPPED_DIVERGED] and steps[1] == 12
    b.close()


def test_batch_close_hands_back_steps_and_state(M):
    """Closing a stepped batch without asking its status leaves each sim
    with the right step count and current buffer: the sim then equals the
    same steps taken alone."""
    shape = (16, 16, 64)
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=64, ny=16, nz=16, A=0.02)
    rR, rB, u = cg_droplet_case(shape, 26)
    _, solo = gpu_run(M, p, rR, rB, u, 13)
    s = M.Sim(p)
    s.init_equilibrium(rR, rB, u)
    b = M.Batch([s], [13])
    b.step(5, use_graph=False)
    b.step(10, use_graph=False)
    torch_sync()
    b.close()
    assert s.observables()["step"] == 13
    assert np.array_equal(s.export_f().cpu().numpy(), solo)


def test_import_export_round_trip(M):
    shape = (8, 8, 32)
    for prec in (0, 1):
        p = M.make_params(lattice=M.D3Q19, precision=prec, nx=32, ny=8, nz=8)
        rR, rB, u = cg_droplet_case(shape, 24)
        s = M.Sim(p)
        s.init_equilibrium(rR, rB, u)
        f = s.export_f()
        s.import_f(f)
        assert (s.export_f() == f).all()


# --------------------------------------------------------------------------
# Batched stepping: bitwise the same as solo, with and without graphs
# --------------------------------------------------------------------------
def test_batch_invariance_bitwise(M):
    cases = [
        (M.make_params(lattice=M.D2Q9, precision=M.FP32, nx=48, ny=40, nz=1, A=0.02), (1, 40, 48), 30),
        (M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=24, ny=20, nz=16, A=0.01), (16, 20, 24), 45),
        (M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=32, ny=16, nz=16, A=0.03, rho0_B=0.1),
         (16, 16, 32), 20),
        (M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=16, ny=16, nz=16, G_RB=1.2),
         (16, 16, 16), 33),
        (M.make_params(lattice=M.D3Q19, precision=M.FP64, nx=20, ny=12, nz=10, A=0.02, bc=(1, 0, 2)),
         (10, 12, 20), 25),
    ]
    inits = []
    for i, (p, shape, _) in enumerate(cases):
        lat = p["lattice"]
        rR, rB, u = cg_droplet_case(shape, 30 + i, gamma=p["rho0_R"] / p["rho0_B"], lattice=lat)
        inits.append((rR, rB, u))
    solo = []
    for (p, shape, n), (rR, rB, u) in zip(cases, inits):
        _, f = gpu_run(M, p, rR, rB, u, n, kernel=1)
        solo.append(f)
    for use_graph in (False, True):
        say(f"[batch] use_graph={use_graph}")
        sims = []
        for (p, shape, n), (rR, rB, u) in zip(cases, inits):
            s = M.Sim(dict(p, kernel=1))
            s.init_equilibrium(rR, rB, u)
            sims.append(s)
        b = M.Batch(sims, [n for (_, _, n) in cases])
        for _ in range(10):
            b.step(7, use_graph=use_graph)
        st, steps = b.status()
        assert st == [M.DONE] * len(cases)
        assert steps == [n for (_, _, n) in cases]
        b.close()
        for s, f in zip(sims, solo):
            assert np.array_equal(s.export_f().cpu().numpy(), f)


def test_batch_one_pass_bitwise(M):
    """Batched one-pass columns (64 x 8, 64 x 4 in FP64 and mixed precision)
    beside batched two-pass sims (ny not a multiple of the column height,
    repulsion, pinned two-pass, D2Q9) in the same batch: every sim ends
    bitwise equal to its solo two-pass run; every precision, all three
    models, walls and outflow, periodic and bounded sims of one group, nx a
    multiple of 64 or not (masked last column where at least 3/4 of the
    columns' lanes hold nodes: 48, 52, 100, 112, 120 and 200 = 3 x 64 + 8; two-pass
    below that: 3, 40, 130; 96 x 4 columns at nx = 96, except FP64 and the mixed
    colour gradient, which take a 64-wide and a masked column), so up to six
    launches of the one-pass kernel per group, z-chunks with a shorter last
    chunk (nz = 101 is prime: every chunk length above one leaves a
    remainder)."""
    def sc_mp(shape):
        a, b = inputs.droplet(shape, 3.0, 1.9, 0.12)
        return a + b, None, None

    D3, F, T = M.D3Q19, M.KERNEL_FUSED, M.KERNEL_TWO_PASS
    cases = [  # params, fields, steps, expected batched kernel
        (M.make_params(lattice=D3, precision=M.FP32, nx=64, ny=16, nz=20, A=0.02), None, 23, F),
        (M.make_params(lattice=D3, precision=M.FP64, nx=64, ny=12, nz=101, A=0.02, bc=(1, 0, 2)), None, 17, F),
        (M.make_params(lattice=D3, precision=M.FP16, nx=64, ny=8, nz=16, A=0.02, bc=(0, 1, 0)), None, 21, F),
        (M.make_params(lattice=D3, precision=M.MIXED, nx=128, ny=16, nz=16, A=0.02, rho0_B=0.01), None, 19, F),
        (M.make_params(lattice=D3, precision=M.MIXED, nx=64, ny=12, nz=20, A=0.02, rho0_B=0.01, bc=(1, 1, 2)),
         None, 16, F),
        (M.make_params(lattice=D3, precision=M.MIXED, nx=64, ny=6, nz=8, A=0.02, rho0_B=0.01), None, 12, T),
        (M.make_params(lattice=D3, precision=M.MIXED, nx=40, ny=10, nz=12, A=0.02, rho0_B=0.01, bc=(1, 0, 2)),
         None, 14, T),
        (M.make_params(lattice=D3, model=M.SC_MC, precision=M.MIXED, nx=64, ny=8, nz=16, G_RB=1.2), None, 22, F),
        (M.make_params(lattice=D3, model=M.SC_MP, precision=M.FP32, nx=64, ny=8, nz=24, G=-5.0, rho0_R=1.9,
                       rho0_B=0.12), "scmp", 25, F),
        (M.make_params(lattice=D3, model=M.SC_MC, precision=M.FP32, nx=64, ny=8, nz=16, G_RB=1.2,
                       bc=(2, 0, 1)), None, 27, F),
        (M.make_params(lattice=D3, precision=M.FP32, nx=40, ny=16, nz=16, A=0.01), None, 29, T),
        (M.make_params(lattice=D3, precision=M.FP32, nx=130, ny=8, nz=12, A=0.01, bc=(1, 0, 2)), None, 11, T),
        (M.make_params(lattice=D3, precision=M.FP32, nx=3, ny=8, nz=9, A=0.01), None, 9, T),
        (M.make_params(lattice=D3, precision=M.FP32, nx=120, ny=8, nz=12, A=0.01, bc=(1, 0, 2)), None, 11, F),
        (M.make_params(lattice=D3, precision=M.FP32, nx=200, ny=8, nz=6, A=0.01), None, 9, F),
        (M.make_params(lattice=D3, precision=M.FP64, nx=100, ny=8, nz=10, A=0.02, bc=(0, 1, 0)), None, 10, F),
        (M.make_params(lattice=D3, precision=M.MIXED, nx=100, ny=8, nz=12, A=0.02, rho0_B=0.01), None, 12, F),
        (M.make_params(lattice=D3, precision=M.FP16, nx=52, ny=8, nz=10, A=0.02, bc=(2, 0, 1)), None, 8, F),
        (M.make_params(lattice=D3, precision=M.FP32, nx=96, ny=8, nz=12, A=0.01), None, 10, F),
        (M.make_params(lattice=D3, precision=M.FP32, nx=96, ny=12, nz=10, A=0.01, bc=(1, 1, 2)), None, 9, F),
        (M.make_params(lattice=D3, precision=M.FP16, nx=96, ny=4, nz=14, A=0.02, bc=(0, 1, 0)), None, 8, F),
        (M.make_params(lattice=D3, precision=M.MIXED, nx=96, ny=8, nz=10, A=0.02, rho0_B=0.01), None, 11, F),
        (M.make_params(lattice=D3, model=M.SC_MC, precision=M.MIXED, nx=96, ny=8, nz=12, G_RB=1.2,
                       bc=(1, 0, 2)), None, 9, F),
        (M.make_params(lattice=D3, precision=M.FP64, nx=96, ny=8, nz=8, A=0.02), None, 7, F),
        (M.make_params(lattice=D3, model=M.SC_MP, precision=M.FP32, nx=48, ny=8, nz=16, G=-5.0, rho0_R=1.9,
                       rho0_B=0.12), "scmp", 13, F),
        (M.make_params(lattice=D3, model=M.SC_MC, precision=M.FP64, nx=112, ny=8, nz=10, G_RB=1.2,
                       bc=(1, 1, 1)), None, 7, F),
        (M.make_params(lattice=D3, precision=M.FP32, nx=64, ny=6, nz=16, A=0.01), None, 13, T),
        (M.make_params(lattice=D3, precision=M.FP32, nx=64, ny=12, nz=16, A=0.01), None, 14, T),
        (M.make_params(lattice=D3, precision=M.FP32, nx=64, ny=8, nz=16, A=0.02, Pi=0.01), None, 15, T),
        (M.make_params(lattice=D3, precision=M.FP32, nx=64, ny=8, nz=16, A=0.02, kernel=T), None, 18, T),
        (M.make_params(lattice=M.D2Q9, precision=M.FP32, nx=64, ny=32, nz=1, A=0.02), None, 31, T),
    ]
    inits = []
    for i, (p, kind, _, _) in enumerate(cases):
        shape = (p["nz"], p["ny"], p["nx"])
        if kind == "scmp":
            inits.append(sc_mp(shape))
        else:
            inits.append(cg_droplet_case(shape, 50 + i, gamma=p["rho0_R"] / p["rho0_B"], lattice=p["lattice"]))
    solo = [gpu_run(M, p, *ini, n, kernel=1)[1] for (p, _, n, _), ini in zip(cases, inits)]
    for use_graph in (False, True):
        say(f"[batch one-pass] use_graph={use_graph}")
        sims = []
        for (p, _, _, _), (rR, rB, u) in zip(cases, inits):
            s = M.Sim(p)
            s.init_equilibrium(rR, rB, u)
            sims.append(s)
        b = M.Batch(sims, [n for (_, _, n, _) in cases])
        assert b.kernels() == [k for (_, _, _, k) in cases]
        for _ in range(5):
            b.step(7, use_graph=use_graph)
        st, steps = b.status()
        b.close()
        assert st == [M.DONE] * len(cases)
        assert steps == [n for (_, _, n, _) in cases]
        for i, (s, f) in enumerate(zip(sims, solo)):
            assert np.array_equal(s.export_f().cpu().numpy(), f), f"case {i}"
            s.close()


def test_batch_graph_replays_match_eager(M):
    """The K-step graph of a batch (one-pass and two-pass groups, walls and
    outflow, side-stream branches) replayed several times, with unrelated
    eager device work and synchronisations between the replays, matches the
    same batch stepped without a graph: equal step counts after every replay
    and, at the end (members of a live batch cannot be read), equal
    populations bit for bit; a wrong replay would leave its mark on the
    final state."""
    import torch
    specs = [
        dict(lattice=M.D3Q19, precision=M.FP32, nx=64, ny=16, nz=12, A=0.02),
        dict(lattice=M.D3Q19, precision=M.FP32, nx=40, ny=12, nz=10, A=0.02, bc=(1, 0, 2)),
        dict(lattice=M.D3Q19, precision=M.MIXED, nx=64, ny=8, nz=8, A=0.02, rho0_B=0.05),
        dict(lattice=M.D2Q9, precision=M.FP64, nx=48, ny=40, nz=1, A=0.02, bc=(0, 1, 0)),
    ]
    def make():
        sims = []
        for i, kw in enumerate(specs):
            p = M.make_params(**kw)
            shape = (p["nz"], p["ny"], p["nx"])
            rR, rB, u = cg_droplet_case(shape, 70 + i, gamma=p["rho0_R"] / p["rho0_B"], lattice=p["lattice"])
            s = M.Sim(p)
            s.init_equilibrium(rR, rB, u)
            sims.append(s)
        return sims
    ga, eb = make(), make()
    A = M.Batch(ga, [10 ** 6] * len(ga))
    B = M.Batch(eb, [10 ** 6] * len(eb))
    scratch = torch.randn(1 << 20, device="cuda")
    for it in range(4):
        A.step(9, use_graph=True)
        B.step(9, use_graph=False)
        scratch = torch.sin(scratch) * 1.0001      # unrelated eager work between replays
        torch.cuda.synchronize()
        sa, na = A.status()
        sb, nb = B.status()
        assert sa == sb == [M.RUNNING] * len(specs) and na == nb == [9 * (it + 1)] * len(specs)
    A.close()
    B.close()
    for i, (a, b) in enumerate(zip(ga, eb)):
        assert np.array_equal(a.export_f().cpu().numpy(), b.export_f().cpu().numpy()), i


def test_solo_steps_captured_in_a_graph(M):
    """mclbm_step with check_every = 0 captured into a HIP graph (an even
    number of steps, after one eager step) and replayed several times, with
    unrelated eager work and synchronisations between the replays, matches
    the same sim stepped eagerly, bit for bit after every replay: one-pass
    D3Q19 (full and masked columns, walls and outflow) and two-pass D2Q9."""
    import torch
    specs = [
        dict(lattice=M.D3Q19, precision=M.FP32, nx=64, ny=16, nz=12, A=0.02, kernel=M.KERNEL_FUSED),
        dict(lattice=M.D3Q19, precision=M.FP32, nx=40, ny=16, nz=10, A=0.02, bc=(1, 0, 2),
             kernel=M.KERNEL_FUSED),
        dict(lattice=M.D2Q9, precision=M.FP64, nx=48, ny=40, nz=1, A=0.02, bc=(0, 1, 0),
             kernel=M.KERNEL_TWO_PASS),
    ]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for i, kw in enumerate(specs):
            say("graph capture case", i, kw)
            p = M.make_params(**kw)
            shape = (p["nz"], p["ny"], p["nx"])
            rR, rB, u = cg_droplet_case(shape, 90 + i, lattice=p["lattice"])
            a, b = M.Sim(p), M.Sim(p)
            a.init_equilibrium(rR, rB, u)
            b.init_equilibrium(rR, rB, u)
            assert a.kernel_used() == kw["kernel"]
            a.step(1)
            b.step(1)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
                a.step(4)
            scratch = torch.randn(1 << 20, device="cuda")
            for it in range(3):
                g.replay()
                b.step(4)
                scratch = torch.sin(scratch) * 1.0001
                torch.cuda.synchronize()
                fa = a.export_f().cpu().numpy()
                fb = b.export_f().cpu().numpy()
                assert np.array_equal(fa, fb), (i, it)
            assert np.isfinite(fa).all()
            del g
            a.close()
            b.close()


def test_side_stream_sim_outputs_ordered_with_caller(M):
    """A sim on a side stream with many steps still queued: moments, export
    and checkpoint read from the caller's (default) stream right away equal
    the same reads taken after the side stream has drained, and an import
    from the default stream is seen by the side stream."""
    import torch
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=128, ny=64, nz=64, A=0.02)
    shape = (64, 64, 128)
    rR, rB, u = cg_droplet_case(shape, 95)
    s = torch.cuda.Stream()
    a = M.Sim(p, stream=s)
    a.init_equilibrium(rR, rB, u)
    a.step(60)                                  # queued on the side stream
    rho_now = a.moments()[0].cpu().numpy()      # default stream
    f_now = a.export_f().cpu().numpy()
    ck, n = a.checkpoint()
    ck_now = ck.cpu().numpy()
    s.synchronize()
    with torch.cuda.stream(s):
        rho_late = a.moments()[0].cpu().numpy()
        f_late = a.export_f().cpu().numpy()
    assert np.array_equal(rho_now, rho_late) and np.array_equal(f_now, f_late)
    assert n == 60 and np.array_equal(ck_now, a.checkpoint()[0].cpu().numpy())
    g = torch.from_numpy(f_late).cuda() * 1.0   # produced on the default stream
    a.import_f(g)
    assert np.array_equal(a.export_f().cpu().numpy(), f_late)
    a.close()


def test_batch_stops_diverged_member(M):
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=16, ny=16, nz=16, A=0.02)
    shape = (16, 16, 16)
    rR, rB, u = cg_droplet_case(shape, 40)
    good, bad = M.Sim(p), M.Sim(p)
    good.init_equilibrium(rR, rB, u)
    bad.init_equilibrium(rR, rB, u)
    f = bad.export_f()
    f[1, 0, 3, 3, 3] = float("inf")
    bad.import_f(f)
    b = M.Batch([good, bad], [30, 30])
    b.step(10)
    b.step(10)
    b.step(10)
    st, steps = b.status()
    assert st == [M.DONE, M.STOPPED_DIVERGED]
    assert steps[0] == 30 and steps[1] == 1


def test_kernel_used_reports_the_dispatch(M):
    """mclbm_kernel_used: fused for D3Q19 when 4 divides ny (any nx) and for
    D2Q9 from 2^19 nodes (any size when requested), two-pass otherwise (D3Q19
    with ny % 4 != 0, the repulsion force, small D2Q9 boxes, forced
    two-pass)."""
    def used(**kw):
        s = M.Sim(M.make_params(**kw))
        k = s.kernel_used()
        s.close()
        return k
    d3 = dict(lattice=M.D3Q19, nx=64, ny=16, nz=8)
    assert used(precision=M.FP32, **d3) == M.KERNEL_FUSED
    assert used(precision=M.MIXED, **d3) == M.KERNEL_FUSED
    assert used(precision=M.FP16, **d3) == M.KERNEL_FUSED
    assert used(precision=M.FP64, **d3) == M.KERNEL_FUSED
    assert used(precision=M.FP64, lattice=M.D3Q19, nx=64, ny=18, nz=8) == M.KERNEL_TWO_PASS
    assert used(precision=M.FP32, kernel=M.KERNEL_TWO_PASS, **d3) == M.KERNEL_TWO_PASS
    assert used(precision=M.FP32, lattice=M.D3Q19, nx=40, ny=16, nz=8) == M.KERNEL_FUSED
    assert used(precision=M.FP32, lattice=M.D3Q19, nx=64, ny=14, nz=8) == M.KERNEL_TWO_PASS
    assert used(precision=M.FP32, lattice=M.D2Q9, nx=1024, ny=512, nz=1) == M.KERNEL_FUSED
    assert used(precision=M.FP64, lattice=M.D2Q9, nx=1000, ny=700, nz=1) == M.KERNEL_FUSED
    # small 2-D boxes: the automatic choice is two-pass, the one-pass kernel on request
    assert used(precision=M.FP32, lattice=M.D2Q9, nx=512, ny=512, nz=1) == M.KERNEL_TWO_PASS
    assert used(precision=M.FP32, lattice=M.D2Q9, nx=64, ny=64, nz=1, kernel=M.KERNEL_FUSED) == M.KERNEL_FUSED
    assert used(precision=M.FP32, lattice=M.D2Q9, nx=2048, ny=2048, nz=1, Pi=0.01) == M.KERNEL_TWO_PASS
