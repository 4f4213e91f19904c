"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/mclbm.h, and its host-side logic (defaults, validation,
layout sizes, sigma <-> A of Eq. sigmaA) behaves as documented."""
import ctypes
import math
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mclbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mclbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def M():
    import paper_2110_05197_amd as M
    M.lib()
    return M


def test_library_exports_every_declared_function(M):
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(M.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_status_strings(M):
    assert M.version() == (2, 0)
    L = M.lib()
    for s in (0, 1, -1, -2, -3, -4):
        assert L.mclbm_status_str(s)
    assert L.mclbm_status_str(99) == b"unknown status"


def test_defaults(M):
    p = M.params_default(M.D3Q19, M.CG)
    assert p["abi_version"] == 3 and p["beta"] == 0.7 and p["alpha_B"] == 0.2 and p["conserve_mass"] == 0
    assert (p["nx"], p["ny"], p["nz"]) == (64, 64, 64)
    assert M.params_default(M.D2Q9, M.CG)["nz"] == 1


def test_sigma_round_trip_eq_sigmaA(M):
    """sigma = 4A/(9 omega_eff) with omega_eff = 2/(6 nu + 1) at rho^N = 0."""
    p = M.make_params(lattice=M.D3Q19, tau_R=1.0, tau_B=0.55)
    p = M.params_from_sigma(p, 0.05)
    nuR, nuB = 0.5 / 3, 0.05 / 3
    nu = 1 / (0.5 / nuR + 0.5 / nuB)
    om = 2 / (6 * nu + 1)
    assert math.isclose(p["A"], 9 * 0.05 * om / 4, rel_tol=1e-14)
    assert math.isclose(M.sigma_from_params(p), 0.05, rel_tol=1e-14)
    # equal taus: sigma = 4A/(9 omega) with omega = 1/tau
    q = M.make_params(A=0.01, tau_R=1.0, tau_B=1.0)
    assert math.isclose(M.sigma_from_params(q), 4 * 0.01 / 9, rel_tol=1e-14)


@pytest.mark.parametrize("lattice,model,prec,expect", [
    (1, 0, 1, 2 * 2 * 19 * 4),   # D3Q19 CG FP32: 304 B per update
    (1, 0, 0, 2 * 2 * 19 * 8),
    (1, 0, 3, 2 * 2 * 19 * 2),
    (0, 0, 1, 2 * 2 * 9 * 4),
    (1, 1, 1, 2 * 1 * 19 * 4),
])
def test_bytes_per_update(M, lattice, model, prec, expect):
    p = M.make_params(lattice=lattice, model=model, precision=prec, nz=1 if lattice == 0 else 64)
    assert M.bytes_per_update(p) == expect


def test_state_bytes_layout(M):
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=32, ny=16, nz=8)
    N = 32 * 16 * 8
    align = lambda b: (b + 255) // 256 * 256
    S, w, arrays = M.population_stride(p)
    assert (w, arrays) == (4, 38)
    assert S * w == align(N * 4) + 256   # small lattices: 256-byte rounding plus 256 B
    f = arrays * S * w
    field = 3 * N * 4
    assert M.state_bytes(p) == 2 * align(f) + align(field)
    p_rep = dict(p, Pi=0.01)
    assert M.state_bytes(p_rep) == 2 * align(f) + align(field) + align(3 * N * 4)


@pytest.mark.parametrize("lattice,model,prec,shape,word,arrays", [
    (1, 0, 1, (256, 256, 256), 4, 38), (1, 0, 0, (128, 128, 512), 8, 38), (1, 0, 3, (160, 160, 160), 4, 19),
    (1, 1, 3, (256, 256, 256), 2, 19), (0, 0, 1, (1, 4096, 4096), 4, 18), (1, 0, 2, (384, 96, 96), 4, 38)])
def test_population_stride_padding(M, lattice, model, prec, shape, word, arrays):
    """Population arrays of 8 MB and more start 256 KB + 256 B past a 1 MB
    boundary of the previous array's end, so that no two arrays of a buffer
    start a multiple of a large power of two apart (a 256^3 FP32 array is
    exactly 64 MB)."""
    nz, ny, nx = shape
    p = M.make_params(lattice=lattice, model=model, precision=prec, nx=nx, ny=ny, nz=nz)
    S, w, a = M.population_stride(p)
    assert (w, a) == (word, arrays)
    N = nx * ny * nz
    b = N * w
    assert b >= 8 << 20
    assert S * w == (b + (1 << 20) - 1) // (1 << 20) * (1 << 20) + (256 << 10) + 256
    assert (S * w) % (1 << 20) == (256 << 10) + 256


@pytest.mark.parametrize("bad", [
    dict(tau_R=0.5), dict(tau_B=0.4), dict(beta=1.5), dict(rho0_B=2.0), dict(alpha_B=1.0),
    dict(nx=1), dict(nz=1), dict(bc=(0, 3, 0)), dict(precision=7), dict(abi_version=9), dict(conserve_mass=2),
    dict(kernel=5), dict(A=-1.0),
])
def test_validation_rejects(M, bad):
    p = M.make_params(lattice=M.D3Q19, **bad)
    with pytest.raises(M.MclbmError) as e:
        M.state_bytes(p)
    assert e.value.status == -1


def test_unsupported_combinations(M):
    with pytest.raises(M.MclbmError) as e:
        M.state_bytes(M.make_params(lattice=M.D3Q19, model=M.SC_MP, Pi=0.01))
    assert e.value.status == -2
    # fused needs no repulsion, and on D3Q19 ny % 4 == 0 (any nx: the last
    # column in x is masked); D2Q9 takes any size
    assert M.state_bytes(M.make_params(lattice=M.D2Q9, nz=1, nx=70, ny=45, kernel=M.KERNEL_FUSED)) > 0
    with pytest.raises(M.MclbmError) as e:
        M.state_bytes(M.make_params(lattice=M.D2Q9, nz=1, Pi=0.01, kernel=M.KERNEL_FUSED))
    assert e.value.status == -2
    with pytest.raises(M.MclbmError):
        M.state_bytes(M.make_params(lattice=M.D3Q19, nx=64, ny=30, kernel=M.KERNEL_FUSED))
    assert M.state_bytes(M.make_params(lattice=M.D3Q19, nx=40, ny=12, kernel=M.KERNEL_FUSED)) > 0
    with pytest.raises(M.MclbmError):
        M.state_bytes(M.make_params(lattice=M.D3Q19, nx=64, ny=18, precision=M.FP64,
                                    kernel=M.KERNEL_FUSED))
    with pytest.raises(M.MclbmError):
        M.state_bytes(M.make_params(lattice=M.D3Q19, nx=64, ny=32, Pi=0.01, kernel=M.KERNEL_FUSED))
    for prec in (M.FP64, M.FP32, M.MIXED, M.FP16):
        assert M.state_bytes(M.make_params(lattice=M.D3Q19, nx=64, ny=32, precision=prec,
                                           kernel=M.KERNEL_FUSED)) > 0


def test_node_count_limit(M):
    """The step kernels use 32-bit node offsets: 2^31 nodes or more are
    refused (EUNSUPPORTED) before any memory is asked for, also for storage
    small enough to fit in HBM (FP16 single-component D2Q9 at 2^31 nodes is
    about 150 GB with both buffers)."""
    for kw in (dict(lattice=M.D3Q19, nx=2048, ny=1024, nz=1024),
               dict(lattice=M.D2Q9, model=M.SC_MP, precision=M.FP16, nx=65536, ny=32768, nz=1)):
        with pytest.raises(M.MclbmError) as e:
            M.state_bytes(M.make_params(**kw))
        assert e.value.status == -2
    assert M.state_bytes(M.make_params(lattice=M.D3Q19, nx=2048, ny=1024, nz=1023)) > 0


def test_d2q9_rejects_z_boundaries(M):
    with pytest.raises(M.MclbmError):
        M.state_bytes(M.make_params(lattice=M.D2Q9, nz=1, bc=(0, 0, 1)))


def test_single_hip_runtime_when_library_loads_first():
    """Loading the library before anything else imports torch must not map a
    second HIP runtime (a second runtime sees no device)."""
    import subprocess
    code = ("import paper_2110_05197_amd as M; M.lib(); "
            "maps = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def test_interface_observables_reject_bad_arguments_without_a_device(M):
    """The interface observables validate their arguments on the host (no
    device work): NULL simulation -> EINVAL."""
    L = M.lib()
    n = ctypes.c_int32()
    a = ctypes.c_double()
    sizes = (ctypes.c_int64 * 4)()
    pos = (ctypes.c_double * 4)()
    assert L.mclbm_interface_crossings(None, 0, 0, 0, pos, 4, ctypes.byref(n)) == -1
    assert L.mclbm_plane_area(None, 0, 0, ctypes.byref(a)) == -1
    assert L.mclbm_droplets(None, 4, ctypes.byref(n), sizes) == -1


def test_multirange_argument_rules(M):
    """Multirange couplings need the two-component Shan-Chen model (EINVAL),
    D3Q19 (EUNSUPPORTED on D2Q9) and the two-pass kernels (EUNSUPPORTED when
    the fused kernel is requested); with all four zero nothing changes."""
    mr = dict(Ga_R=-9.0, Ga_B=-8.0, Gr_R=8.1, Gr_B=7.1, psi_rho0=0.83, rho0_X=0.83)
    with pytest.raises(M.MclbmError) as e:
        M.state_bytes(M.make_params(lattice=M.D3Q19, model=M.CG, **mr))
    assert e.value.status == -1
    with pytest.raises(M.MclbmError) as e:
        M.state_bytes(M.make_params(lattice=M.D2Q9, nz=1, model=M.SC_MC, **mr))
    assert e.value.status == -2
    with pytest.raises(M.MclbmError) as e:
        M.state_bytes(M.make_params(lattice=M.D3Q19, model=M.SC_MC, kernel=M.KERNEL_FUSED, **mr))
    assert e.value.status == -2
    p = M.make_params(lattice=M.D3Q19, model=M.SC_MC, precision=M.FP32, nx=32, ny=16, nz=8, **mr)
    q = dict(p, Ga_R=0.0, Ga_B=0.0, Gr_R=0.0, Gr_B=0.0)
    N = 32 * 16 * 8
    # two more stencil fields (psi of each species) with the multirange forces
    assert M.state_bytes(p) - M.state_bytes(q) == (4 - 2) * N * 4
