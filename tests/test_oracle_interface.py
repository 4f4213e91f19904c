"""Pins of the oracle's interface observables (radius along a line by linear
interpolation, plane phase area, connected droplets) against constructions
whose answers are known exactly and against scipy's labelling."""
import numpy as np
import pytest


def fields_from_rhoN(rhoN):
    """Two-component fields of total density 1 with the given rho^N."""
    rR = 0.5 * (1.0 + rhoN)
    return rR, 1.0 - rR


@pytest.mark.parametrize("bc", [0, 1])
def test_crossings_exact_on_a_linear_profile(orc, bc):
    """rho^N = 0.02 (x - 10.3) on 40 nodes: the crossing is 10.3 (linear
    interpolation is exact on a linear field); on a periodic axis the wrap
    segment (x = 39 -> 0) adds 39 + 0.574 / (0.574 + 0.206)."""
    nx = 40
    x = np.arange(nx, dtype=float)
    rhoN = np.broadcast_to(0.02 * (x - 10.3), (1, 4, nx)).copy()
    rR, rB = fields_from_rhoN(rhoN)
    p = orc.make_params(lattice=0, nx=nx, ny=4, nz=1, bc=(bc, 0, 0))
    f = orc.init_equilibrium(p, rR, rB)
    pos, n = orc.interface_crossings(p, f, 0, 2, 0)
    if bc == 0:
        a, b = 0.02 * (39 - 10.3), 0.02 * (0 - 10.3)
        assert n == 2
        assert pos[0] == pytest.approx(10.3, abs=1e-12)
        assert pos[1] == pytest.approx(39 + a / (a - b), abs=1e-12)
    else:
        assert n == 1 and pos[0] == pytest.approx(10.3, abs=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_crossings_line_addressing_d3q19(orc, axis):
    """A slab |s - c| < 3.5, c = (n - 1)/2 + 0.25, along each axis of a
    16x12x10 box; the line is taken through (c1, c2) = the other coordinates
    in increasing axis order, and only that line carries the slab (elsewhere
    the box is blue), so a wrong line reads no crossings."""
    shape = (10, 12, 16)  # (nz, ny, nx)
    n_ax = shape[::-1][axis]
    s = np.arange(n_ax, dtype=float)
    cen = (n_ax - 1) / 2 + 0.25
    prof = np.clip((3.5 - np.abs(s - cen)) / 2.0, -0.9, 0.9)
    rhoN = np.full(shape, -0.9)
    other = [a for a in range(3) if a != axis]
    c = {other[0]: 3, other[1]: 5}
    sl = [slice(None)] * 3
    for a in other:
        sl[2 - a] = c[a]
    rhoN[tuple(sl)] = prof
    rR, rB = fields_from_rhoN(rhoN)
    p = orc.make_params(lattice=1, nx=16, ny=12, nz=10)
    f = orc.init_equilibrium(p, rR, rB)
    pos, n = orc.interface_crossings(p, f, axis, 3, 5)
    assert n == 2
    assert pos[0] == pytest.approx(cen - 3.5, abs=1e-12)
    assert pos[1] == pytest.approx(cen + 3.5, abs=1e-12)
    _, n_other = orc.interface_crossings(p, f, axis, 4, 5)
    assert n_other == 0


@pytest.mark.parametrize("model", [0, 1])
def test_plane_area_is_the_plane_sum(orc, model):
    rng = np.random.default_rng(5)
    shape = (12, 10, 8)
    if model == 0:
        rR = rng.uniform(0.1, 1.0, shape)
        rB = rng.uniform(0.1, 1.0, shape)
        p = orc.make_params(lattice=1, nx=8, ny=10, nz=12)
        f = orc.init_equilibrium(p, rR, rB)
        frac = 0.5 * (1 + (rR - rB) / (rR + rB))
    else:
        rho = rng.uniform(0.1, 2.0, shape)
        p = orc.make_params(lattice=1, model=1, nx=8, ny=10, nz=12, G=-5.0, rho0_R=1.9,
                            rho0_B=0.1)
        f = orc.init_equilibrium(p, rho, None)
        frac = (rho >= 1.0).astype(float)
    for axis, pos in ((0, 3), (1, 7), (2, 5)):
        expect = frac.take(pos, axis=2 - axis).sum()
        assert orc.plane_area(p, f, axis, pos) == pytest.approx(expect, rel=1e-12, abs=1e-12)


def _partition(labels):
    """Components as a set of frozensets of flat node indices."""
    flat = labels.ravel()
    out = {}
    for n, l in enumerate(flat):
        if l >= 0:
            out.setdefault(l, []).append(n)
    return {frozenset(v) for v in out.values()}


def test_components_match_scipy_between_walls(orc):
    """Random blobs in a 28x24x20 box with walls on every axis: the oracle's
    face-connected components equal scipy.ndimage.label's, and each label is
    the smallest node index of its component."""
    from scipy import ndimage
    rng = np.random.default_rng(11)
    shape = (20, 24, 28)
    noise = ndimage.uniform_filter(rng.normal(size=shape), size=3, mode="constant")
    mask = noise > 0.15
    rR, rB = fields_from_rhoN(np.where(mask, 0.8, -0.8))
    p = orc.make_params(lattice=1, nx=28, ny=24, nz=20, bc=(1, 1, 1))
    f = orc.init_equilibrium(p, rR, rB)
    count, labels = orc.label_components(p, f)
    ref, nref = ndimage.label(mask)
    assert count == nref > 10
    assert _partition(labels) == _partition(np.where(ref > 0, ref, -1))
    for comp in _partition(labels):
        assert labels.ravel()[min(comp)] == min(comp)


def _sphere_mask(shape, centre, r):
    """Periodic ball; shape in (.., y, x) order, centre in (x, y, ..) order."""
    coords = np.indices(shape)[::-1]
    dims = shape[::-1]
    d2 = 0.0
    for v, c, n in zip(coords, centre, dims):
        dv = np.abs(v - c)
        d2 = d2 + np.minimum(dv, n - dv) ** 2     # minimum image
    return d2 <= r * r


def test_components_periodic_wrap_and_face_adjacency(orc):
    shape = (16, 16, 16)
    # a sphere centred on a corner of the periodic box is one droplet, split
    # into the 8 octant pieces when the faces are walls
    m = _sphere_mask(shape, (0.0, 0.0, 0.0), 4.5)
    rR, rB = fields_from_rhoN(np.where(m, 0.8, -0.8))
    p = orc.make_params(lattice=1, nx=16, ny=16, nz=16)
    f = orc.init_equilibrium(p, rR, rB)
    c, lab = orc.label_components(p, f)
    assert c == 1 and (lab >= 0).sum() == m.sum()
    pw = orc.make_params(lattice=1, nx=16, ny=16, nz=16, bc=(1, 1, 1))
    assert orc.label_components(pw, orc.init_equilibrium(pw, rR, rB))[0] == 8
    # two cubes that share only an edge are two droplets (face adjacency)
    m = np.zeros(shape, bool)
    m[2:5, 2:5, 2:5] = True
    m[2:5, 5:8, 5:8] = True
    rR, rB = fields_from_rhoN(np.where(m, 0.8, -0.8))
    c, lab = orc.label_components(p, orc.init_equilibrium(p, rR, rB))
    assert c == 2 and sorted(np.unique(lab[lab >= 0], return_counts=True)[1]) == [27, 27]


def test_components_d2q9_disks(orc):
    """Three disks on a periodic 64x48 plane, one across the x faces."""
    shape = (1, 48, 64)
    m = np.zeros(shape, bool)
    for centre, r in (((10.0, 10.0), 5.0), ((40.0, 30.0), 6.0), ((63.5, 20.0), 4.0)):
        m[0] |= _sphere_mask((48, 64), centre, r)
    rR, rB = fields_from_rhoN(np.where(m, 0.8, -0.8))
    p = orc.make_params(lattice=0, nx=64, ny=48, nz=1)
    c, lab = orc.label_components(p, orc.init_equilibrium(p, rR, rB))
    assert c == 3 and (lab >= 0).sum() == m.sum()
