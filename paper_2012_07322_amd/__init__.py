"""Python binding of libgmunu (the MI355X GRMHD finite-volume step).

Argument marshalling only: every step runs in the HIP kernels of
``csrc/gmunu.hip`` behind the C ABI of ``include/gmunu.h``.  PyTorch
provides device memory and the stream.  There is no CPU fallback: if the
library is not built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libgmunu.so")

CART, CYL, SPH = 0, 1, 2
PERIODIC, OUTFLOW, REFLECT, AXIS, CENTER, NONE = 0, 1, 2, 3, 4, 5
FLAG_ATMO, FLAG_EPS_CLAMP, FLAG_V_CLAMP = 1, 2, 4
FLAG_FATAL_RHO, FLAG_FATAL_EPS, FLAG_FATAL_V, FLAG_NOCONV = 8, 16, 32, 64

ERRORS = {-1: "invalid argument", -2: "null pointer", -3: "misaligned pointer", -4: "HIP error",
          -5: "out of device memory"}


class GridDesc(ctypes.Structure):
    """Mirror of gmunu_grid_desc."""
    _fields_ = [
        ("ndim", ctypes.c_int), ("coord", ctypes.c_int), ("n", ctypes.c_int * 3), ("ng", ctypes.c_int),
        ("xmin", ctypes.c_double * 3), ("dx", ctypes.c_double * 3),
        ("bc", (ctypes.c_int * 2) * 3),
        ("gamma", ctypes.c_double),
        ("rho_atmo", ctypes.c_double), ("k_atmo", ctypes.c_double), ("gamma_atmo", ctypes.c_double),
        ("rho_low_factor", ctypes.c_double), ("alpha_bh", ctypes.c_double),
        ("rho_max", ctypes.c_double), ("eps_max", ctypes.c_double), ("w_max", ctypes.c_double),
        ("c2p_maxit", ctypes.c_int), ("c2p_tol", ctypes.c_double),
        ("rk", ctypes.c_int),
    ]


DEFAULTS = dict(ng=2, gamma=5.0 / 3.0, rho_atmo=1e-12, k_atmo=100.0, gamma_atmo=2.0,
                rho_low_factor=100.0, alpha_bh=1e-2, rho_max=math.inf, eps_max=math.inf,
                w_max=1e3, c2p_maxit=200, c2p_tol=1e-15, rk=3)

_lib = None
_P = ctypes.c_void_p


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgmunu is not built ({LIB_PATH}); run paper_2012_07322_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        I, D = ctypes.c_int, ctypes.c_double
        L.gmunu_create.argtypes = [_P, ctypes.POINTER(_P)]
        L.gmunu_destroy.argtypes = [_P]
        L.gmunu_ntot.argtypes = [_P]
        L.gmunu_ntot.restype = ctypes.c_long
        L.gmunu_prim2con.argtypes = [_P, _P, _P, _P, _P]
        L.gmunu_c2p.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.gmunu_fill_ghosts.argtypes = [_P, _P, _P]
        L.gmunu_rhs.argtypes = [_P, _P, _P, _P, _P]
        L.gmunu_cfl_dt.argtypes = [_P, _P, _P, D, D, _P, _P, _P]
        L.gmunu_rk_stage.argtypes = [_P, I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.gmunu_step.argtypes = [_P, _P, _P, _P, _P, D, D, _P, _P, _P, _P, _P]
        L.gmunu_profile.argtypes = [_P, I, I]
        L.gmunu_profile_read.argtypes = [_P, _P, _P]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed: {ERRORS.get(rc, rc)}")


def make_desc(p: dict) -> GridDesc:
    q = dict(DEFAULTS)
    q.update(p)
    d = GridDesc()
    d.ndim, d.coord, d.ng = int(q["ndim"]), int(q["coord"]), int(q["ng"])
    for a in range(3):
        d.n[a] = int(q["n"][a])
        d.xmin[a] = float(q["xmin"][a])
        d.dx[a] = float(q["dx"][a])
        d.bc[a][0] = int(q["bc"][a][0])
        d.bc[a][1] = int(q["bc"][a][1])
    for k in ("gamma", "rho_atmo", "k_atmo", "gamma_atmo", "rho_low_factor", "alpha_bh", "rho_max", "eps_max",
              "w_max", "c2p_tol"):
        setattr(d, k, float(q[k]))
    d.c2p_maxit, d.rk = int(q["c2p_maxit"]), int(q["rk"])
    return d


def _ptr(t, what, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A grid context: geometry tables and scratch on the current device."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self.desc = make_desc(params)
        h = _P()
        _check(lib().gmunu_create(ctypes.byref(self.desc), ctypes.byref(h)), "gmunu_create")
        self._h = h
        d = self.desc
        g = [d.ng if a < d.ndim else 0 for a in range(3)]
        self.shape = (d.n[2] + 2 * g[2], d.n[1] + 2 * g[1], d.n[0] + 2 * g[0])
        self.ntot = int(lib().gmunu_ntot(h))
        self.nstages = d.rk

    def close(self):
        if getattr(self, "_h", None):
            lib().gmunu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, t, nv, what):
        if t is None:
            return None
        if tuple(t.shape) != (nv,) + self.shape:
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {(nv,) + self.shape}")
        return _ptr(t, what)

    def empty_state(self, nv=8, device="cuda"):
        return torch.zeros((nv,) + self.shape, dtype=torch.float64, device=device)

    def prim2con(self, prim, metric, q=None):
        q = self.empty_state() if q is None else q
        _check(lib().gmunu_prim2con(self._h, self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"),
                                    self._chk(q, 8, "q"), _stream()), "gmunu_prim2con")
        return q

    def c2p(self, q, metric, prim, flags=None, nfatal=None):
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        if flags is not None and tuple(flags.shape) != self.shape:
            raise ValueError("flags shape")
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_c2p(self._h, self._chk(q, 8, "q"), self._chk(metric, 5, "metric"),
                               self._chk(prim, 8, "prim"), fp, npn, _stream()), "gmunu_c2p")
        return prim

    def fill_ghosts(self, prim):
        _check(lib().gmunu_fill_ghosts(self._h, self._chk(prim, 8, "prim"), _stream()), "gmunu_fill_ghosts")
        return prim

    def rhs(self, prim, metric, out=None):
        out = self.empty_state() if out is None else out
        _check(lib().gmunu_rhs(self._h, self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"),
                               self._chk(out, 8, "dqdt"), _stream()), "gmunu_rhs")
        return out

    def cfl_dt(self, prim, metric, cfl, t_end=math.inf, t_dev=None, dt_dev=None):
        dt_dev = torch.zeros(1, dtype=torch.float64, device=prim.device) if dt_dev is None else dt_dev
        _check(lib().gmunu_cfl_dt(self._h, self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"), cfl, t_end,
                                  _ptr(t_dev, "t"), _ptr(dt_dev, "dt"), _stream()), "gmunu_cfl_dt")
        return dt_dev

    def rk_stage(self, stage, dt_dev, q_n, q_s, q_out, prim_in, prim_out, metric, flags=None, nfatal=None):
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_rk_stage(self._h, stage, _ptr(dt_dev, "dt"), self._chk(q_n, 8, "q_n"),
                                    self._chk(q_s, 8, "q_s"), self._chk(q_out, 8, "q_out"),
                                    self._chk(prim_in, 8, "prim_in"), self._chk(prim_out, 8, "prim_out"),
                                    self._chk(metric, 5, "metric"), fp, npn, _stream()), "gmunu_rk_stage")

    KERNELS = ("stage", "c2p", "ghosts", "cfl", "other")

    def profile(self, enable=True, max_launches=8192):
        _check(lib().gmunu_profile(self._h, 1 if enable else 0, max_launches), "gmunu_profile")

    def profile_read(self):
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_long * 5)()
        _check(lib().gmunu_profile_read(self._h, ms, cnt), "gmunu_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNELS)}

    def step(self, q_n, q_s, prim, metric, cfl, t_end, t_dev, dt_dev, flags=None, nfatal=None):
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_step(self._h, self._chk(q_n, 8, "q_n"), self._chk(q_s, 8, "q_s"),
                                self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"), cfl, t_end,
                                _ptr(t_dev, "t"), _ptr(dt_dev, "dt"), fp, npn, _stream()), "gmunu_step")


# ------------------------------------------------------------------- batch

class BlockSpec(ctypes.Structure):
    """Mirror of gmunu_block."""
    _fields_ = [("desc", GridDesc), ("q_n", _P), ("q_s", _P), ("prim", _P), ("metric", _P), ("flags", _P),
                ("group", ctypes.c_int)]


def _batch_sigs(L):
    I, D = ctypes.c_int, ctypes.c_double
    L.gmunu_batch_create.argtypes = [I, I, ctypes.c_long, ctypes.POINTER(_P)]
    L.gmunu_batch_destroy.argtypes = [_P]
    L.gmunu_batch_set_block.argtypes = [_P, I, ctypes.POINTER(BlockSpec)]
    L.gmunu_batch_clear_block.argtypes = [_P, I]
    L.gmunu_batch_set_group.argtypes = [_P, I, D, D, I]
    L.gmunu_batch_commit.argtypes = [_P, _P]
    L.gmunu_batch_autotune.argtypes = [_P, _P]
    L.gmunu_batch_init.argtypes = [_P, _P, I, _P]
    L.gmunu_batch_step.argtypes = [_P, D, _P, I, _P]
    L.gmunu_batch_times.argtypes = [_P, _P, _P, _P, _P]
    L.gmunu_batch_info.argtypes = [_P, _P, _P]


def state_shape(p: dict):
    d = make_desc(p)
    g = [d.ng if a < d.ndim else 0 for a in range(3)]
    return (d.n[2] + 2 * g[2], d.n[1] + 2 * g[1], d.n[0] + 2 * g[0])


class Arena:
    """One device allocation sliced into 256-byte aligned views."""

    def __init__(self, ndoubles, device="cuda"):
        self.buf = torch.empty(int(ndoubles), dtype=torch.float64, device=device)
        self.off = 0

    @staticmethod
    def size_of(shapes):
        tot = 0
        for s in shapes:
            n = 1
            for x in s:
                n *= x
            tot += (n + 31) // 32 * 32
        return tot

    def take(self, shape):
        n = 1
        for x in shape:
            n *= x
        v = self.buf[self.off:self.off + n].view(shape)
        self.off += (n + 31) // 32 * 32
        return v


class Batch:
    """Many grids advanced together (gmunu_batch_*): blocks in slots, groups
    sharing a time step, persistent kernels, a graph-captured step."""

    def __init__(self, max_blocks, max_groups, max_items):
        L = lib()
        if not hasattr(L, "_batch_sigs_set"):
            _batch_sigs(L)
            L._batch_sigs_set = True
        h = _P()
        _check(L.gmunu_batch_create(max_blocks, max_groups, max_items, ctypes.byref(h)), "gmunu_batch_create")
        self._h = h
        self.max_blocks, self.max_groups = max_blocks, max_groups
        self.keep = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().gmunu_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_block(self, slot, params, q_n, q_s, prim, metric, group, flags=None):
        shp = state_shape(params)
        for t, nv, nm in ((q_n, 8, "q_n"), (q_s, 8, "q_s"), (prim, 8, "prim"), (metric, 5, "metric")):
            if tuple(t.shape) != (nv,) + shp:
                raise ValueError(f"{nm} has shape {tuple(t.shape)}, expected {(nv,) + shp}")
        spec = BlockSpec()
        spec.desc = make_desc(params)
        spec.q_n, spec.q_s, spec.prim = _ptr(q_n, "q_n"), _ptr(q_s, "q_s"), _ptr(prim, "prim")
        spec.metric = _ptr(metric, "metric")
        spec.flags = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        spec.group = group
        _check(lib().gmunu_batch_set_block(self._h, slot, ctypes.byref(spec)), "gmunu_batch_set_block")
        self.keep[slot] = (q_n, q_s, prim, metric, flags)

    def clear_block(self, slot):
        _check(lib().gmunu_batch_clear_block(self._h, slot), "gmunu_batch_clear_block")
        self.keep.pop(slot, None)

    def set_group(self, group, t, t_end, max_steps=0):
        _check(lib().gmunu_batch_set_group(self._h, group, t, t_end, max_steps), "gmunu_batch_set_group")

    def commit(self):
        _check(lib().gmunu_batch_commit(self._h, _stream()), "gmunu_batch_commit")

    def autotune(self):
        _check(lib().gmunu_batch_autotune(self._h, _stream()), "gmunu_batch_autotune")

    def init(self, slots=None):
        if slots is None:
            _check(lib().gmunu_batch_init(self._h, None, 0, _stream()), "gmunu_batch_init")
        else:
            arr = (ctypes.c_int * len(slots))(*slots)
            _check(lib().gmunu_batch_init(self._h, arr, len(slots), _stream()), "gmunu_batch_init")

    def step(self, cfl, nfatal=None, use_graph=True):
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_batch_step(self._h, cfl, npn, 1 if use_graph else 0, _stream()), "gmunu_batch_step")

    def times(self, with_steps=False):
        import numpy as np
        t = np.zeros(self.max_groups)
        dt = np.zeros(self.max_groups)
        ns = np.zeros(self.max_groups, dtype=np.int32)
        _check(lib().gmunu_batch_times(self._h, t.ctypes.data_as(_P), dt.ctypes.data_as(_P),
                                       ns.ctypes.data_as(_P), _stream()), "gmunu_batch_times")
        return (t, dt, ns) if with_steps else (t, dt)

    def info(self):
        import numpy as np
        items = np.zeros(3, dtype=np.int64)
        var = np.zeros(self.max_blocks, dtype=np.int32)
        _check(lib().gmunu_batch_info(self._h, items.ctypes.data_as(_P), var.ctypes.data_as(_P)), "gmunu_batch_info")
        return items, var
