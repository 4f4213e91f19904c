"""Seeded synthetic initial fields shaped like the paper's test cases.

This module holds geometry and random draws only (droplets, ellipsoids,
ligaments, jets, slabs, shear waves); none of the lattice Boltzmann
arithmetic.  Both the HIP path and the oracle consume the arrays it returns,
so it imports neither of them.

Every profile is a diffuse interface phi = tanh(d / width) with d the signed
distance to the interface (positive inside the red fluid), and
    rho_R = rho0_R (1 + phi) / 2,   rho_B = rho0_B (1 - phi) / 2.
Arrays are float64 with shape (nz, ny, nx); velocities have shape
(3, nz, ny, nx).  Random numbers come from numpy.random.default_rng(seed).
"""
from __future__ import annotations

import numpy as np


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _min_image(d, n, periodic):
    if periodic:
        return d - n * np.round(d / n)
    return d


def fields_from_distance(d, rho0_R, rho0_B, width=2.0):
    phi = np.tanh(d / width)
    return rho0_R * 0.5 * (1.0 + phi), rho0_B * 0.5 * (1.0 - phi)


def droplet(shape, radius, rho0_R=1.0, rho0_B=1.0, center=None, width=2.0, periodic=True):
    """Sphere (or disk when nz == 1) centred at ``center``; default centre is
    ((n-1)/2) per axis, which keeps the box's mirror symmetries."""
    nz, ny, nx = shape
    if center is None:
        center = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    x, y, z = _grid(shape)
    dx = _min_image(x - center[0], nx, periodic)
    dy = _min_image(y - center[1], ny, periodic)
    dz = _min_image(z - center[2], nz, periodic) if nz > 1 else 0.0 * z
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    return fields_from_distance(radius - r, rho0_R, rho0_B, width)


def ellipsoid(shape, semi_axes, rho0_R=1.0, rho0_B=1.0, center=None, width=2.0):
    """Ellipsoid with the given semi-axes (ax, ay, az); the signed distance is
    approximated by (1 - s) * mean semi-axis with s the scaled radius."""
    nz, ny, nx = shape
    if center is None:
        center = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    x, y, z = _grid(shape)
    ax, ay, az = semi_axes
    s = np.sqrt(((x - center[0]) / ax) ** 2 + ((y - center[1]) / ay) ** 2
                + ((z - center[2]) / az) ** 2)
    d = (1.0 - s) * (ax + ay + az) / 3.0
    return fields_from_distance(d, rho0_R, rho0_B, width)


def perturbed_ellipsoid(shape, semi_axes, seed, jitter=1.0, **kw):
    """Ellipsoid whose semi-axes are each shifted by U[-jitter, jitter]."""
    rng = np.random.default_rng(seed)
    ax = [a + rng.uniform(-jitter, jitter) for a in semi_axes]
    return ellipsoid(shape, ax, **kw), ax


def random_droplets(shape, count, rmin, rmax, seed, rho0_R=1.0, rho0_B=1.0, width=2.0,
                    gap=4.0, max_tries=100000):
    """``count`` non-overlapping spheres with radii U[rmin, rmax] at uniform
    positions, placed by rejection in a periodic box (minimum image)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    placed = []
    tries = 0
    while len(placed) < count and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        c = (rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz))
        ok = True
        for (c2, r2) in placed:
            d = [c[a] - c2[a] for a in range(3)]
            d = [d[a] - n * round(d[a] / n) for a, n in enumerate((nx, ny, nz))]
            if np.sqrt(sum(v * v for v in d)) < r + r2 + gap:
                ok = False
                break
        if ok:
            placed.append((c, r))
    # signed distance to the nearest sphere, evaluated only in a box around
    # each sphere (beyond r + 12 width the profile is saturated to 1e-10)
    dmax = np.full(shape, -12.0 * width)
    for (c, r) in placed:
        reach = r + 12.0 * width
        idx = []
        for a, n in enumerate((nx, ny, nz)):
            lo = int(np.floor(c[a] - reach))
            q = np.arange(lo, int(np.ceil(c[a] + reach)) + 1)
            if len(q) >= n:
                q = np.arange(n)
            idx.append(q)
        qx, qy, qz = idx
        dx = _min_image(qx % nx - c[0], nx, True)
        dy = _min_image(qy % ny - c[1], ny, True)
        dz = _min_image(qz % nz - c[2], nz, True)
        d = r - np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        sub = np.ix_(qz % nz, qy % ny, qx % nx)
        dmax[sub] = np.maximum(dmax[sub], d)
    rR, rB = fields_from_distance(dmax, rho0_R, rho0_B, width)
    return rR, rB, placed


def droplet_pair(shape, radius, separation, speed, rho0_R=1.0, rho0_B=1.0, width=2.0):
    """Two equal spheres on the x axis through the box centre, centres
    ``separation`` apart, moving towards each other at ``speed``: u_x is
    +speed inside the left droplet and -speed inside the right one, each
    weighted by that droplet's red fraction (1 + phi) / 2.  Returns
    (rho_R, rho_B, u)."""
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    r2 = (y - cy) ** 2 + (z - cz) ** 2
    dl = radius - np.sqrt((x - (cx - separation / 2.0)) ** 2 + r2)
    dr = radius - np.sqrt((x - (cx + separation / 2.0)) ** 2 + r2)
    rR, rB = fields_from_distance(np.maximum(dl, dr), rho0_R, rho0_B, width)
    u = np.zeros((3,) + tuple(shape))
    u[0] = speed * 0.5 * (1.0 + np.tanh(dl / width)) - speed * 0.5 * (1.0 + np.tanh(dr / width))
    return rR, rB, u


def jet(shape, radius, wavelength, amplitude, phase=0.0, rho0_R=1.0, rho0_B=1.0, width=2.0):
    """Cylinder along z with radius R (1 + a sin(2 pi z / lambda + phase))."""
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    rloc = radius * (1.0 + amplitude * np.sin(2 * np.pi * z / wavelength + phase))
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return fields_from_distance(rloc - r, rho0_R, rho0_B, width)


def ligament(shape, radius, length, rho0_R=1.0, rho0_B=1.0, width=2.0, axis=2):
    """Capsule: a cylinder of total length ``length`` (caps included) with
    hemispherical caps, centred in the box along ``axis`` (0 = x, 2 = z)."""
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    ctr = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    coords = (x - ctr[0], y - ctr[1], z - ctr[2])
    half = max(length / 2.0 - radius, 0.0)
    a = np.clip(coords[axis], -half, half)
    d2 = (coords[axis] - a) ** 2
    for k in range(3):
        if k != axis:
            d2 = d2 + coords[k] ** 2
    return fields_from_distance(radius - np.sqrt(d2), rho0_R, rho0_B, width)


def slab(shape, thickness, rho0_R=1.0, rho0_B=1.0, axis=0, width=2.0):
    """Red slab of the given thickness, centred along ``axis`` (flat interfaces)."""
    n = shape[::-1][axis]
    x, y, z = _grid(shape)
    q = (x, y, z)[axis] - (n - 1) / 2.0
    return fields_from_distance(thickness / 2.0 - np.abs(q), rho0_R, rho0_B, width)


def shear_wave(shape, amplitude, axis_u=0, axis_k=1):
    """Velocity u_{axis_u} = a sin(2 pi q / n) along axis_k."""
    n = shape[::-1][axis_k]
    x, y, z = _grid(shape)
    q = (x, y, z)[axis_k]
    u = np.zeros((3,) + tuple(shape))
    u[axis_u] = amplitude * np.sin(2 * np.pi * q / n)
    return u


def noise(shape, amplitude, seed):
    """Uniform noise U[-a, a] (for perturbing states in tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=shape)
