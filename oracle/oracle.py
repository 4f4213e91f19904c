"""ctypes front end of the FP64 CPU oracle (``mclbm_oracle.c``).

Test infrastructure only: the tests, the package entry point's smoke check
and the benchmark's CPU-baseline leg use it; the product never does.  It
imports nothing from the HIP package.

Parameters travel as a plain ``dict`` with the field names of the C struct
(the same dict the HIP binding takes).  Arrays are NumPy float64 in the
layout documented at the top of the C file:
``f[k, i, z, y, x]`` and ``v[d, z, y, x]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mclbm_oracle.c")
_LIB = os.path.join(_HERE, "libmclbm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("model", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3), ("enhanced_eq", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("rho0_R", ctypes.c_double), ("rho0_B", ctypes.c_double),
        ("tau_R", ctypes.c_double), ("tau_B", ctypes.c_double),
        ("A", ctypes.c_double), ("beta", ctypes.c_double), ("alpha_B", ctypes.c_double),
        ("g_min", ctypes.c_double), ("G", ctypes.c_double), ("psi_rho0", ctypes.c_double),
        ("G_RB", ctypes.c_double), ("rho0_X", ctypes.c_double),
        ("Pi", ctypes.c_double), ("chi", ctypes.c_double),
        ("Ga_R", ctypes.c_double), ("Ga_B", ctypes.c_double),
        ("Gr_R", ctypes.c_double), ("Gr_B", ctypes.c_double),
    ]


DEFAULTS = dict(lattice=1, model=0, nx=8, ny=8, nz=8, bc=(0, 0, 0), enhanced_eq=1,
                rho0_R=1.0, rho0_B=1.0, tau_R=1.0, tau_B=1.0, A=0.01, beta=0.7,
                alpha_B=0.2, g_min=1e-8, G=0.0, psi_rho0=1.0, G_RB=0.0, rho0_X=1.0,
                Pi=0.0, chi=1.0, Ga_R=0.0, Ga_B=0.0, Gr_R=0.0, Gr_B=0.0)

_lib = None
_lib_path = None   # None: the parity build; else a timing build (use_library)


def build_timing(directory: str) -> str:
    """The same source built for timing on the host that runs it (gcc -O3
    -march=native, OpenMP; contraction off as in the parity build) into
    `directory`; the benchmark's CPU baseline times this copy."""
    path = os.path.join(directory, "libmclbm_oracle_timing.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-ffp-contract=off", "-std=c11",
                           "-shared", "-fPIC", "-o", path, _SRC, "-lm"])
    return path


def use_library(path: str) -> None:
    """Load the oracle from `path` (a build_timing copy) from now on."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path


def lib():
    global _lib
    if _lib is None:
        path = _lib_path
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        L.orc_lattice_tables.argtypes = [ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_int32), dp, dp, dp, dp, dp]
        L.orc_cg_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp,
                                         ctypes.c_double, ctypes.c_int, dp]
        L.orc_gradient.argtypes = [pp, dp, dp]
        L.orc_moments.argtypes = [pp, dp, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [pp, dp, dp, dp, dp]
        L.orc_collide.argtypes = [pp, dp, dp]
        L.orc_stream.argtypes = [pp, dp, dp]
        L.orc_repulsion_force.argtypes = [pp, dp, dp]
        L.orc_run.argtypes = [pp, dp, ctypes.c_int64]
        L.orc_observables.argtypes = [pp, dp, dp]
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_phase_indicator.argtypes = [pp, dp, dp]
        L.orc_interface_crossings.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                              ctypes.c_int]
        L.orc_interface_crossings.restype = ctypes.c_int
        L.orc_plane_area.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int]
        L.orc_plane_area.restype = ctypes.c_double
        L.orc_label_components.argtypes = [pp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_label_components.restype = ctypes.c_int64
        L.orc_belts_table.argtypes = [ctypes.POINTER(ctypes.c_int32), dp, dp]
        L.orc_belts_table.restype = ctypes.c_int
        L.orc_sc_forces.argtypes = [pp, dp, dp, dp]
        _lib = L
    return _lib


def make_params(**kw) -> dict:
    p = dict(DEFAULTS)
    p.update(kw)
    return p


def _struct(p: dict) -> Params:
    s = Params()
    for k, v in DEFAULTS.items():
        val = p.get(k, v)
        if k == "bc":
            s.bc[:] = [int(b) for b in val]
        else:
            setattr(s, k, val)
    return s


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def Q_of(p: dict) -> int:
    return 9 if p["lattice"] == 0 else 19


def ncomp(p: dict) -> int:
    return 1 if p["model"] == 1 else 2


def shape(p: dict):
    return (p["nz"], p["ny"], p["nx"])


def lattice_tables(lattice: int, alpha: float):
    Q = 9 if lattice == 0 else 19
    c = np.zeros((Q, 3), dtype=np.int32)
    arr = [np.zeros(Q) for _ in range(5)]
    lib().orc_lattice_tables(lattice, alpha, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             *[_ptr(a) for a in arr])
    w, B, psi, xi, phi = arr
    return dict(c=c, w=w, B=B, psi=psi, xi=xi, phi=phi)


def cg_equilibrium(lattice, rho_k, alpha_k, u, grad_k, nubar, enhanced=1):
    Q = 9 if lattice == 0 else 19
    out = np.zeros(Q)
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.ascontiguousarray(grad_k, dtype=np.float64)
    lib().orc_cg_equilibrium(lattice, rho_k, alpha_k, _ptr(u), _ptr(g), nubar, enhanced, _ptr(out))
    return out


def gradient(p: dict, X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.zeros((3,) + shape(p))
    s = _struct(p)
    lib().orc_gradient(ctypes.byref(s), _ptr(X), _ptr(out))
    return out


def init_equilibrium(p: dict, rhoR, rhoB, u=None) -> np.ndarray:
    rhoR = np.ascontiguousarray(rhoR, dtype=np.float64)
    rhoB = np.ascontiguousarray(rhoB if rhoB is not None else np.zeros_like(rhoR), dtype=np.float64)
    f = np.zeros((ncomp(p), Q_of(p)) + shape(p))
    s = _struct(p)
    up = None
    if u is not None:
        u = np.ascontiguousarray(u, dtype=np.float64)
        up = _ptr(u)
    rc = lib().orc_init_equilibrium(ctypes.byref(s), _ptr(rhoR), _ptr(rhoB), up, _ptr(f))
    if rc:
        raise MemoryError("oracle init failed")
    return f


def run(p: dict, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance a copy of ``f`` by ``nsteps`` steps and return it."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    s = _struct(p)
    if lib().orc_run(ctypes.byref(s), _ptr(f), int(nsteps)):
        raise MemoryError("oracle run failed")
    return f


def collide(p: dict, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    s = _struct(p)
    if lib().orc_collide(ctypes.byref(s), _ptr(f), _ptr(out)):
        raise MemoryError("oracle collide failed")
    return out


def stream(p: dict, fpost: np.ndarray) -> np.ndarray:
    fpost = np.ascontiguousarray(fpost, dtype=np.float64)
    out = np.zeros_like(fpost)
    s = _struct(p)
    lib().orc_stream(ctypes.byref(s), _ptr(fpost), _ptr(out))
    return out


def repulsion_force(p: dict, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros((3,) + shape(p))
    s = _struct(p)
    if lib().orc_repulsion_force(ctypes.byref(s), _ptr(f), _ptr(out)):
        raise MemoryError("oracle force failed")
    return out


def moments(p: dict, f: np.ndarray):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rR = np.zeros(shape(p))
    rB = np.zeros(shape(p))
    j = np.zeros((3,) + shape(p))
    s = _struct(p)
    lib().orc_moments(ctypes.byref(s), _ptr(f), _ptr(rR), _ptr(rB), _ptr(j))
    return rR, rB, j


OBS_KEYS = ("mass_R", "mass_B", "mom_x", "mom_y", "mom_z", "ekin", "umax", "rho_in", "rho_out",
            "eps_used", "red_volume", "n_in", "n_out", "diverged")


def observables(p: dict, f: np.ndarray) -> dict:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(len(OBS_KEYS))
    s = _struct(p)
    lib().orc_observables(ctypes.byref(s), _ptr(f), _ptr(out))
    return dict(zip(OBS_KEYS, out.tolist()))


def set_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def phase_indicator(p: dict, f: np.ndarray) -> np.ndarray:
    """rho^N (two components) or rho - (rho0_R + rho0_B)/2 (SC multiphase), (nz, ny, nx)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros((p["nz"], p["ny"], p["nx"]))
    lib().orc_phase_indicator(ctypes.byref(_struct(p)), _ptr(f), _ptr(out))
    return out


def interface_crossings(p: dict, f: np.ndarray, axis: int, c1: int, c2: int, max_out: int = 64):
    """Interpolated interface positions along a lattice line (ascending)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(max_out)
    n = lib().orc_interface_crossings(ctypes.byref(_struct(p)), _ptr(f), axis, c1, c2, _ptr(out),
                                      max_out)
    return out[:min(n, max_out)].copy(), n


def plane_area(p: dict, f: np.ndarray, axis: int, pos: int) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    return float(lib().orc_plane_area(ctypes.byref(_struct(p)), _ptr(f), axis, pos))


def label_components(p: dict, f: np.ndarray):
    """(count, labels (nz, ny, nx) int64: smallest node index of the component, -1 outside)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    labels = np.zeros((p["nz"], p["ny"], p["nx"]), dtype=np.int64)
    n = lib().orc_label_components(ctypes.byref(_struct(p)), _ptr(f),
                                   labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return int(n), labels


def belts_table():
    """The multirange neighbourhood: (c (n, 3) int, p (n,), w (n,))."""
    c = np.zeros((92, 3), dtype=np.int32)
    p = np.zeros(92)
    w = np.zeros(92)
    n = lib().orc_belts_table(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(p), _ptr(w))
    return c[:n].copy(), p[:n].copy(), w[:n].copy()


def sc_forces(p: dict, f: np.ndarray):
    """Two-component Shan-Chen forces on each colour, (3, nz, ny, nx) each."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    shape = (3, p["nz"], p["ny"], p["nx"])
    FR, FB = np.zeros(shape), np.zeros(shape)
    lib().orc_sc_forces(ctypes.byref(_struct(p)), _ptr(f), _ptr(FR), _ptr(FB))
    return FR, FB
