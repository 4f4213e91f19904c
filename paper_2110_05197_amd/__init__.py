"""MI355X two-component lattice Boltzmann (colour gradient / Shan-Chen).

Thin ctypes binding of ``libmclbm.so`` (declared in ``include/mclbm.h``):
argument marshalling only.  Every step of the method runs in the library's
HIP kernels; PyTorch supplies device memory and the stream.  If the library
is not built, every entry point raises -- there is no CPU fallback.

Parameters are a plain dict with the field names of ``mclbm_params``;
arrays use the layout of the header: ``f[k, i, z, y, x]``, ``u[d, z, y, x]``.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["MclbmError", "Sim", "Batch", "lib", "make_params", "params_default",
           "params_from_sigma", "sigma_from_params", "state_bytes", "bytes_per_update", "population_stride",
           "version",
           "D2Q9", "D3Q19", "CG", "SC_MP", "SC_MC", "FP64", "FP32", "MIXED", "FP16",
           "PERIODIC", "WALL", "OUTFLOW", "KERNEL_AUTO", "KERNEL_TWO_PASS", "KERNEL_FUSED",
           "OK", "DIVERGED", "RUNNING", "DONE", "STOPPED_DIVERGED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmclbm.so")

OK, DIVERGED = 0, 1
D2Q9, D3Q19 = 0, 1
CG, SC_MP, SC_MC = 0, 1, 2
FP64, FP32, MIXED, FP16 = 0, 1, 2, 3
PERIODIC, WALL, OUTFLOW = 0, 1, 2
KERNEL_AUTO, KERNEL_TWO_PASS, KERNEL_FUSED = 0, 1, 2
RUNNING, DONE, STOPPED_DIVERGED = 0, 1, 2
ABI_VERSION = 3


class MclbmError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("lattice", ctypes.c_int32), ("model", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("bc", ctypes.c_int32 * 3), ("enhanced_eq", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("rho0_R", ctypes.c_double), ("rho0_B", ctypes.c_double), ("tau_R", ctypes.c_double),
        ("tau_B", ctypes.c_double), ("A", ctypes.c_double), ("beta", ctypes.c_double),
        ("alpha_B", ctypes.c_double), ("g_min", ctypes.c_double), ("G", ctypes.c_double),
        ("psi_rho0", ctypes.c_double), ("G_RB", ctypes.c_double), ("rho0_X", ctypes.c_double),
        ("Pi", ctypes.c_double), ("chi", ctypes.c_double),
        ("Ga_R", ctypes.c_double), ("Ga_B", ctypes.c_double),
        ("Gr_R", ctypes.c_double), ("Gr_B", ctypes.c_double),
        ("conserve_mass", ctypes.c_int32),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("mass_R", ctypes.c_double), ("mass_B", ctypes.c_double), ("mom", ctypes.c_double * 3),
        ("ekin", ctypes.c_double), ("umax", ctypes.c_double), ("rho_in", ctypes.c_double),
        ("rho_out", ctypes.c_double), ("eps_used", ctypes.c_double),
        ("red_volume", ctypes.c_double), ("n_in", ctypes.c_double), ("n_out", ctypes.c_double),
        ("diverged", ctypes.c_double), ("step", ctypes.c_int64),
    ]


_lib = None
_vp = ctypes.c_void_p
_P = ctypes.POINTER(Params)


def lib():
    """Load libmclbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2110_05197_amd._build` (no CPU fallback exists)")
        # The library must share the HIP runtime that owns the caller's device
        # memory and streams.  Loading torch first puts its libamdhip64 in the
        # process, and the library's dependency then resolves to that copy;
        # loaded the other way round, two runtimes coexist and the second one
        # sees no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int32
        sigs = {
            "mclbm_version": [ctypes.POINTER(ctypes.c_int32)] * 2,
            "mclbm_params_default": [_P, ctypes.c_int32, ctypes.c_int32],
            "mclbm_params_from_sigma": [_P, ctypes.c_double],
            "mclbm_sigma_from_params": [_P, ctypes.POINTER(ctypes.c_double)],
            "mclbm_state_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
            "mclbm_bytes_per_update": [_P, ctypes.POINTER(ctypes.c_double)],
            "mclbm_population_stride": [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)],
            "mclbm_create": [_P, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
            "mclbm_destroy": [_vp],
            "mclbm_init_equilibrium": [_vp, _vp, _vp, _vp],
            "mclbm_step": [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
            "mclbm_moments": [_vp, _vp, _vp, _vp],
            "mclbm_observables": [_vp, ctypes.POINTER(Obs)],
            "mclbm_export_f": [_vp, _vp],
            "mclbm_import_f": [_vp, _vp],
            "mclbm_checkpoint_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
            "mclbm_checkpoint": [_vp, _vp, ctypes.POINTER(ctypes.c_int64)],
            "mclbm_restore": [_vp, _vp, ctypes.c_int64],
            "mclbm_diverged": [_vp, ctypes.POINTER(ctypes.c_int32)],
            "mclbm_kernel_used": [_vp, ctypes.POINTER(ctypes.c_int32)],
            "mclbm_fused_tile": [_vp] + [ctypes.POINTER(ctypes.c_int32)] * 3,
            "mclbm_interface_crossings": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)],
            "mclbm_interface_crossings_noalloc": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_int32)],
            "mclbm_plane_area": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
            "mclbm_droplets": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int64)],
            "mclbm_batch_create": [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                   _vp, ctypes.POINTER(_vp)],
            "mclbm_batch_step": [_vp, ctypes.c_int32, ctypes.c_int32],
            "mclbm_batch_status": [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)],
            "mclbm_batch_kernels": [_vp, ctypes.POINTER(ctypes.c_int32)],
            "mclbm_batch_destroy": [_vp],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.mclbm_status_str.argtypes = [st]
        L.mclbm_status_str.restype = ctypes.c_char_p
        L.mclbm_last_error.argtypes = []
        L.mclbm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status, where, allow=(OK,)):
    if status in allow:
        return status
    L = lib()
    raise MclbmError(status, where, f"{L.mclbm_status_str(status).decode()}: "
                                    f"{L.mclbm_last_error().decode()}")


def version():
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mclbm_version(ctypes.byref(a), ctypes.byref(b)), "mclbm_version")
    return a.value, b.value


def _to_struct(p: dict) -> Params:
    s = Params()
    _check(lib().mclbm_params_default(ctypes.byref(s), int(p.get("lattice", D3Q19)),
                                      int(p.get("model", CG))), "mclbm_params_default")
    for name, _ in Params._fields_:
        if name in p:
            if name == "bc":
                s.bc[:] = [int(b) for b in p["bc"]]
            else:
                setattr(s, name, p[name])
    return s


def _to_dict(s: Params) -> dict:
    d = {}
    for name, _ in Params._fields_:
        v = getattr(s, name)
        d[name] = tuple(v) if name == "bc" else v
    return d


def params_default(lattice=D3Q19, model=CG) -> dict:
    s = Params()
    _check(lib().mclbm_params_default(ctypes.byref(s), lattice, model), "mclbm_params_default")
    return _to_dict(s)


def make_params(**kw) -> dict:
    """Library defaults for (lattice, model) overridden by ``kw``."""
    d = params_default(kw.get("lattice", D3Q19), kw.get("model", CG))
    d.update(kw)
    return d


def params_from_sigma(p: dict, sigma: float) -> dict:
    s = _to_struct(p)
    _check(lib().mclbm_params_from_sigma(ctypes.byref(s), sigma), "mclbm_params_from_sigma")
    return dict(p, A=s.A)


def sigma_from_params(p: dict) -> float:
    s = _to_struct(p)
    out = ctypes.c_double()
    _check(lib().mclbm_sigma_from_params(ctypes.byref(s), ctypes.byref(out)), "mclbm_sigma_from_params")
    return out.value


def state_bytes(p: dict) -> int:
    s = _to_struct(p)
    out = ctypes.c_size_t()
    _check(lib().mclbm_state_bytes(ctypes.byref(s), ctypes.byref(out)), "mclbm_state_bytes")
    return out.value


def bytes_per_update(p: dict) -> float:
    s = _to_struct(p)
    out = ctypes.c_double()
    _check(lib().mclbm_bytes_per_update(ctypes.byref(s), ctypes.byref(out)), "mclbm_bytes_per_update")
    return out.value


def population_stride(p: dict):
    """(words between population arrays, bytes per word, arrays per buffer)."""
    s = _to_struct(p)
    w, b, a = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mclbm_population_stride(ctypes.byref(s), ctypes.byref(w), ctypes.byref(b), ctypes.byref(a)),
           "mclbm_population_stride")
    return w.value, b.value, a.value


def _torch():
    import torch
    return torch


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Sim:
    """One simulation on caller (torch) memory; mirrors the mclbm_* calls.

    The library enqueues on `stream` (default: the current stream at
    creation).  Tensors passed in or returned are ordered with the caller's
    current stream at the time of the call, whichever stream that is."""

    def __init__(self, params: dict, device="cuda", stream=None):
        torch = _torch()
        self.params = dict(params)
        self._s = _to_struct(self.params)
        self.nbytes = state_bytes(self.params)
        self.device = torch.device(device)
        # 256-byte alignment: allocate slack and offset
        self._buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._buf.data_ptr()) % 256
        self._base = self._buf.data_ptr() + off
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().mclbm_create(ctypes.byref(self._s), ctypes.c_void_p(self._base), self.nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "mclbm_create")
        self._h = h
        p = self.params
        self.Q = 9 if p["lattice"] == D2Q9 else 19
        self.ncomp = 1 if p["model"] == SC_MP else 2
        self.shape = (p["nz"], p["ny"], p["nx"])
        self.N = p["nx"] * p["ny"] * p["nz"]

    def close(self):
        if getattr(self, "_h", None):
            lib().mclbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _after_caller(self):
        """Order the sim's stream after the caller's current stream: the
        library is about to read tensors the caller's stream produced, or to
        write fresh tensors whose memory that stream last used."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _before_caller(self):
        """Order the caller's current stream after the sim's stream: tensors
        the library wrote on its stream are then safe to use on the caller's."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _dev64(self, a, shape):
        torch = _torch()
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        assert tuple(t.shape) == tuple(shape), (t.shape, shape)
        return t

    def init_equilibrium(self, rhoR, rhoB=None, u=None):
        tR = self._dev64(rhoR, self.shape)
        tB = self._dev64(rhoB, self.shape)
        tu = self._dev64(u, (3,) + self.shape)
        self._after_caller()
        _check(lib().mclbm_init_equilibrium(self._h, _dptr(tR), _dptr(tB), _dptr(tu)),
               "mclbm_init_equilibrium")
        self._keep = (tR, tB, tu)   # alive until the stream has consumed them
        self.stream.synchronize()
        self._keep = None

    def step(self, nsteps, check_every=0):
        """Returns (status, steps_done); status OK or DIVERGED."""
        done = ctypes.c_int64()
        st = _check(lib().mclbm_step(self._h, int(nsteps), int(check_every), ctypes.byref(done)),
                    "mclbm_step", allow=(OK, DIVERGED))
        return st, done.value

    def moments(self):
        torch = _torch()
        rR = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        rB = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._after_caller()
        _check(lib().mclbm_moments(self._h, _dptr(rR), _dptr(rB), _dptr(u)), "mclbm_moments")
        self._before_caller()
        return rR, rB, u

    def observables(self) -> dict:
        o = Obs()
        _check(lib().mclbm_observables(self._h, ctypes.byref(o)), "mclbm_observables")
        return dict(mass_R=o.mass_R, mass_B=o.mass_B, mom_x=o.mom[0], mom_y=o.mom[1],
                    mom_z=o.mom[2], ekin=o.ekin, umax=o.umax, rho_in=o.rho_in, rho_out=o.rho_out,
                    eps_used=o.eps_used, red_volume=o.red_volume, n_in=o.n_in, n_out=o.n_out,
                    diverged=o.diverged, step=o.step)

    def export_f(self):
        torch = _torch()
        f = torch.empty((self.ncomp, self.Q) + self.shape, dtype=torch.float64, device=self.device)
        self._after_caller()
        _check(lib().mclbm_export_f(self._h, _dptr(f)), "mclbm_export_f")
        self._before_caller()
        return f

    def import_f(self, f):
        t = self._dev64(f, (self.ncomp, self.Q) + self.shape)
        self._after_caller()
        _check(lib().mclbm_import_f(self._h, _dptr(t)), "mclbm_import_f")
        self.stream.synchronize()

    def checkpoint(self):
        torch = _torch()
        nb = ctypes.c_size_t()
        _check(lib().mclbm_checkpoint_bytes(self._h, ctypes.byref(nb)), "mclbm_checkpoint_bytes")
        buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        step = ctypes.c_int64()
        self._after_caller()
        _check(lib().mclbm_checkpoint(self._h, _dptr(buf), ctypes.byref(step)), "mclbm_checkpoint")
        self._before_caller()
        return buf, step.value

    def restore(self, buf, step):
        self._after_caller()
        _check(lib().mclbm_restore(self._h, _dptr(buf), int(step)), "mclbm_restore")
        self._before_caller()   # buf may be freed or reused on the caller's stream

    def diverged(self) -> bool:
        d = ctypes.c_int32()
        _check(lib().mclbm_diverged(self._h, ctypes.byref(d)), "mclbm_diverged")
        return bool(d.value)

    def interface_crossings(self, axis: int, c1: int, c2: int, max_out: int = 64, noalloc: bool = False):
        """Interpolated interface positions along the lattice line parallel to
        `axis` through (c1, c2) (the other coordinates, in axis order), ascending.
        noalloc: the allocation-free entry point (static device scratch, lines
        of up to 32768 nodes)."""
        out = (ctypes.c_double * max(1, max_out))()
        n = ctypes.c_int32()
        name = "mclbm_interface_crossings_noalloc" if noalloc else "mclbm_interface_crossings"
        _check(getattr(lib(), name)(self._h, axis, c1, c2, out, max_out, ctypes.byref(n)), name)
        return [out[i] for i in range(min(n.value, max_out))], n.value

    def plane_area(self, axis: int, pos: int) -> float:
        a = ctypes.c_double()
        _check(lib().mclbm_plane_area(self._h, axis, pos, ctypes.byref(a)), "mclbm_plane_area")
        return a.value

    def droplets(self, max_out: int = 1024):
        """(number of face-connected inside regions, their node counts, largest first)."""
        sizes = (ctypes.c_int64 * max(1, max_out))()
        n = ctypes.c_int32()
        _check(lib().mclbm_droplets(self._h, max_out, ctypes.byref(n), sizes), "mclbm_droplets")
        return n.value, [sizes[i] for i in range(min(n.value, max_out))]

    def kernel_used(self) -> int:
        """KERNEL_FUSED or KERNEL_TWO_PASS: the step kernel this simulation runs."""
        k = ctypes.c_int32()
        _check(lib().mclbm_kernel_used(self._h, ctypes.byref(k)), "mclbm_kernel_used")
        return k.value

    def fused_tile(self):
        """(tx, ty, planes): the column (or row segment) and march length of one
        block of the one-pass kernel."""
        v = [ctypes.c_int32() for _ in range(3)]
        _check(lib().mclbm_fused_tile(self._h, *[ctypes.byref(x) for x in v]), "mclbm_fused_tile")
        return tuple(x.value for x in v)


class Batch:
    """Sims advanced together (mclbm_batch_*)."""

    def __init__(self, sims, targets, stream=None):
        torch = _torch()
        self.sims = list(sims)
        n = len(self.sims)
        arr = (ctypes.c_void_p * n)(*[s._h.value for s in self.sims])
        tg = (ctypes.c_int64 * n)(*[int(t) for t in targets])
        # graphs cannot be captured on the null stream: default to a stream of
        # our own (default priority)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _check(lib().mclbm_batch_create(arr, n, tg, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(h)), "mclbm_batch_create")
        self._h = h

    def step(self, ksteps, use_graph=True):
        _check(lib().mclbm_batch_step(self._h, int(ksteps), 1 if use_graph else 0), "mclbm_batch_step")

    def status(self):
        n = len(self.sims)
        st = (ctypes.c_int32 * n)()
        steps = (ctypes.c_int64 * n)()
        _check(lib().mclbm_batch_status(self._h, st, steps), "mclbm_batch_status")
        return list(st), list(steps)

    def kernels(self):
        """KERNEL_FUSED or KERNEL_TWO_PASS per sim: the batched kernel it runs."""
        k = (ctypes.c_int32 * len(self.sims))()
        _check(lib().mclbm_batch_kernels(self._h, k), "mclbm_batch_kernels")
        return list(k)

    def close(self):
        if getattr(self, "_h", None):
            lib().mclbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
