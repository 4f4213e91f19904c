"""The allocation-free interface-crossing entry point against the allocating
one, through the C ABI: same positions and counts on two calls in a row
(the second on a shorter line of a smaller simulation), and a line beyond
its static scratch rejected before any device work."""
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


def _sim(M, shape, R, steps):
    nz, ny, nx = shape
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=nx, ny=ny, nz=nz, A=0.02)
    rR, rB = inputs.droplet(shape, R)
    rR = rR * (1 + inputs.noise(shape, 0.01, 5))
    s = M.Sim(p)
    s.init_equilibrium(rR, rB)
    s.step(steps, check_every=steps)
    return s


def test_noalloc_crossings_equal_allocating_ones(M):
    big = _sim(M, (48, 40, 96), 14.0, 30)      # lines of 96, 40 and 48 nodes
    small = _sim(M, (16, 16, 24), 4.0, 20)     # lines of 24 and 16 nodes
    for sim, axis, c1, c2, label in ((big, 0, 20, 24, "first call, 96-node line"),
                                     (small, 1, 12, 8, "second call, 16-node line"),
                                     (big, 2, 48, 20, "third call, 48-node line")):
        say(f"[noalloc] {label}")
        ref, nref = sim.interface_crossings(axis, c1, c2, max_out=16)
        got, ngot = sim.interface_crossings(axis, c1, c2, max_out=16, noalloc=True)
        assert nref >= 2, "the line must cross the droplet"
        assert ngot == nref
        assert np.array_equal(np.array(got), np.array(ref))
    # fewer output slots than crossings: the count stays the full count
    ref, nref = small.interface_crossings(1, 12, 8, max_out=1)
    got, ngot = small.interface_crossings(1, 12, 8, max_out=1, noalloc=True)
    assert (ngot, got) == (nref, ref) and len(got) == 1


def test_noalloc_rejects_lines_beyond_its_scratch(M):
    p = M.make_params(lattice=M.D3Q19, precision=M.FP32, nx=32776, ny=4, nz=2, kernel=M.KERNEL_TWO_PASS)
    s = M.Sim(p)
    s.init_equilibrium(np.ones((2, 4, 32776)), np.zeros((2, 4, 32776)))
    with pytest.raises(M.MclbmError) as e:
        s.interface_crossings(0, 1, 1, noalloc=True)
    assert e.value.status == -2
    assert "32768" in str(e.value)
    # the allocating call serves the same line
    _, n = s.interface_crossings(0, 1, 1)
    assert n == 0
